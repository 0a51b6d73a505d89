// C ABI of the library: context set-up, workspace layout and the entry points
// declared in include/rec.h.  Host code only; every step of the method runs in
// the kernels of score.hip, fields.hip, sort.hip and search.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"

namespace {

inline int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

inline double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Sizes {
  int npl;
  int64_t Mp, m, mcap, max_nnz, wcap, list_cap, cand_cap, ccap, pool_cap, pcap, dcap, sort_cap,
      best_cap, ex_cap;
};

rec_status plan(const rec_config* c, Sizes* z, const char** why) {
  if (c->N < 2 || c->N > (int64_t(1) << 20)) { *why = "N must be in [2, 2^20]"; return REC_E_INVAL; }
  if (c->M < 1 || c->M > 2048) { *why = "M must be in [1, 2048]"; return REC_E_INVAL; }
  if (c->model < 0 || c->model > 2) { *why = "unknown model"; return REC_E_INVAL; }
  if ((c->model == REC_GAUSS) != (c->xtype == REC_X_FP32)) {
    *why = "Gaussian model needs float32 data, Ising/kinetic need int8 +-1";
    return REC_E_INVAL;
  }
  if (c->prec != REC_FP32 && c->prec != REC_FP64) { *why = "unknown precision"; return REC_E_INVAL; }
  int64_t cols = c->model == REC_KINETIC ? c->M + 1 : c->M;
  if (c->ldx < cols) { *why = "ldx smaller than the number of columns"; return REC_E_INVAL; }
  if (!(c->lambda >= 0) || !std::isfinite(c->lambda)) { *why = "lambda must be finite and >= 0"; return REC_E_INVAL; }
  if (!(c->kappa > 0) || !std::isfinite(c->kappa)) { *why = "kappa must be > 0"; return REC_E_INVAL; }
  const int64_t N = c->N;
  // Ising / kinetic rows hold at least 128 samples: the screening
  // contraction takes 128-sample steps, each inside one operand half
  int npl = c->model == REC_GAUSS ? 1 : 2;
  while (64 * npl < c->M) npl *= 2;
  z->npl = npl;
  z->Mp = 64 * (int64_t)npl;
  z->m = std::max<int64_t>(1, (int64_t)std::floor(c->kappa * (double)N + 0.5));
  const int64_t pairs = N * (N - 1) / (c->model == REC_KINETIC ? 1 : 2);
  z->mcap = std::min<int64_t>(pairs, std::max<int64_t>(4 * z->m, 4096));
  z->max_nnz = c->max_nnz > 0 ? c->max_nnz : 64 * N;
  z->wcap = pow2_at_least(2 * z->max_nnz);
  int64_t k0 = std::max<int64_t>(1, std::min<int64_t>((4 * z->mcap + N - 1) / N, N - 1));
  if (c->knn_k_override > 0) k0 = std::min<int64_t>(c->knn_k_override, N - 1);
  z->list_cap = std::max<int64_t>(4 * z->mcap + N, N * k0) + 1024;
  int64_t want = N * std::min<int64_t>(4 * k0 * k0, N - 1);
  want = std::max(want, 2 * z->mcap + N);
  z->cand_cap = std::min<int64_t>(std::max<int64_t>(want, 1 << 16), int64_t(1) << 27);
  // slot words: cache slots + overflow slots must stay below 2^31 (top bit = owner)
  int lc = c->log2_cache;
  if (lc <= 0) {
    // every pair a FindBest call scores, at a load of at most a half where
    // memory allows (about N k^2 per NNDescent level; 1024 N covers it)
    int64_t target = std::min<int64_t>(std::max<int64_t>(4 * z->cand_cap, 1024 * N), 2 * pairs + 1024);
    lc = 16;
    while ((int64_t(1) << lc) < target && lc < 30) ++lc;
  }
  if (lc < 10 || lc > 30) { *why = "log2_cache must be in [10, 30]"; return REC_E_INVAL; }
  z->ccap = int64_t(1) << lc;
  int levels_max = 2;
  for (int64_t v = 1; v < N; v <<= 1) ++levels_max;
  z->pool_cap = 2 * z->mcap * (levels_max + 1) + 1024;
  z->pcap = pow2_at_least(2 * z->pool_cap);
  z->dcap = pow2_at_least(8 * z->mcap + 1024);
  z->ex_cap = std::min<int64_t>(z->cand_cap, int64_t(1) << 24);
  z->sort_cap = std::max({2 * z->max_nnz, z->list_cap, z->pool_cap, z->ex_cap + z->mcap}) + 1024;
  z->best_cap = std::max<int64_t>(z->mcap, 1024);
  return REC_OK;
}

// Carve the workspace; with a.base == nullptr only the size is computed.
void layout(rec_ctx* x, const rec_config* c, const Sizes& z, Arena& a) {
  const int64_t N = c->N;
  const size_t rs = c->prec == REC_FP32 ? 4 : 8;
  const int64_t nsz = N * z.Mp;
  Fields& F = x->F;
  // the +-1 input side carries REC_TAIL_ROWS zero rows past N (a contraction operand)
  F.xs = a.take<int8_t>(c->model == REC_GAUSS ? nsz : (N + REC_TAIL_ROWS) * z.Mp);
  F.ys = c->model == REC_KINETIC ? a.take<int8_t>(nsz) : F.xs;
  F.xf = c->model == REC_GAUSS ? a.take<float>(nsz) : nullptr;
  F.H = a.take<char>(nsz * rs);
  F.T = c->model == REC_GAUSS ? nullptr : (void*)a.take<char>(nsz * rs);
  if (c->model != REC_GAUSS) {
    F.xq = a.take<uint32_t>(N * 64);
    F.yq = c->model == REC_KINETIC ? a.take<uint32_t>(N * 64) : F.xq;
    F.rq = a.take<int8_t>((N + REC_TAIL_ROWS) * z.Mp);
    F.u4 = a.take<uint32_t>(N * rec_u4_words(z.npl) * 64);
  } else {
    F.xq = F.yq = nullptr;
    F.rq = nullptr;
    F.u4 = nullptr;
  }
  F.sq = a.take<double>(N);
  F.theta = a.take<double>(N);
  x->W.keys = a.take<uint64_t>(z.wcap);
  x->W.vals = a.take<double>(z.wcap);
  x->W.mask = (uint64_t)(z.wcap - 1);
  x->W.bloom = a.take<uint32_t>(REC_WBLOOM_WORDS);
  x->row_off = a.take<int64_t>(N + 1);
  x->col = a.take<int32_t>(2 * z.max_nnz);
  x->colw = a.take<double>(2 * z.max_nnz);
  x->wi = a.take<int32_t>(z.max_nnz);
  x->wj = a.take<int32_t>(z.max_nnz);
  x->wv = a.take<double>(z.max_nnz);
  x->counter = a.take<int64_t>(16);
  x->work = a.take<int64_t>(REC_WORK_N * REC_WORK_COPIES);
  x->dscratch = a.take<double>(std::max<int64_t>(N, 1024));
  x->dresult = a.take<double>(16);
  x->cd_acc = a.take<double>(N / 2 + 1);
  x->err_flag = a.take<int32_t>(4);
  for (int b = 0; b < 2; ++b) {
    x->sb.khi[b] = a.take<uint64_t>(z.sort_cap);
    x->sb.klo[b] = a.take<uint64_t>(z.sort_cap);
    x->sb.val[b] = a.take<uint32_t>(z.sort_cap);
  }
  x->sb.hist = a.take<uint32_t>(256 * ((z.sort_cap + 4095) / 4096 + 1));
  x->sb.cap = z.sort_cap;
  x->C.keys = a.take<uint64_t>(z.ccap);
  x->C.vals = a.take<double>(z.ccap);
  x->C.mask = (uint64_t)(z.ccap - 1);
  x->C.ovf = a.take<double>(z.cand_cap);
  x->C.ovf_cap = z.cand_cap;
  x->list_cap = z.list_cap;
  x->Gidx = a.take<int32_t>(z.list_cap);
  x->Gidx2 = a.take<int32_t>(z.list_cap);
  x->Ggain = a.take<double>(z.list_cap);
  x->Ggain2 = a.take<double>(z.list_cap);
  x->S = a.take<int32_t>(N);
  x->S2 = a.take<int32_t>(N);
  x->loc = nullptr;
  x->cnt = a.take<int64_t>(N + 2);
  x->off = a.take<int64_t>(N + 2);
  x->cand_cap = z.cand_cap;
  x->cand_v = a.take<int32_t>(z.cand_cap);
  x->cand_gi = a.take<int32_t>(z.cand_cap);
  x->cand_slot = a.take<uint32_t>(z.cand_cap);
  x->ts_i = a.take<int32_t>(z.cand_cap);
  x->ts_j = a.take<int32_t>(z.cand_cap);
  x->ts_slot = a.take<uint32_t>(z.cand_cap);
  x->inoff = a.take<int64_t>(N + 2);
  x->capcnt = a.take<int32_t>(N);
  x->in_src = a.take<int32_t>(z.list_cap);
  x->dset_keys = a.take<uint64_t>(z.dcap);
  x->dset_mask = (uint64_t)(z.dcap - 1);
  x->pset_keys = a.take<uint64_t>(z.pcap);
  x->pset_mask = (uint64_t)(z.pcap - 1);
  x->pool_cap = z.pool_cap;
  x->pool_hi = a.take<uint64_t>(z.pool_cap);
  x->pool_lo = a.take<uint64_t>(z.pool_cap);
  x->scan_tmp = a.take<int64_t>(2 * N + 4096);
  x->best_cap = z.best_cap;
  x->best_i = a.take<int32_t>(z.best_cap);
  x->best_j = a.take<int32_t>(z.best_cap);
  x->best_g = a.take<double>(z.best_cap);
  x->pred = a.take<int32_t>(2 * z.best_cap);
  x->pend[0] = a.take<int32_t>(z.best_cap);
  x->pend[1] = a.take<int32_t>(z.best_cap);
  x->done = a.take<uint8_t>(z.best_cap);
  x->dw = a.take<double>(z.best_cap);
  x->ready = a.take<int32_t>(z.best_cap);
  x->depth = a.take<int32_t>(z.best_cap);
  x->best_slot = a.take<int64_t>(z.best_cap);
  x->ex_cap = z.ex_cap;
  x->max_nnz = z.max_nnz;
  x->scr_qcap = std::min<int64_t>(z.cand_cap, int64_t(1) << 30);
  x->scr_queue = a.take<uint32_t>(x->scr_qcap);
  {
    const int64_t B = REC_SUR_BATCH, NP = REC_SUR_NPARAM;
    x->sur_pbits = a.take<uint32_t>(z.Mp);
    x->sur_S = a.take<float>(N * REC_SUR_SDIM);
    x->sur_Sb = a.take<__bf16>(N * REC_SUR_SDIM);
    x->sur_par = a.take<float>(NP);
    x->sur_m = a.take<float>(NP);
    x->sur_v = a.take<float>(NP);
    x->sur_g = a.take<float>(NP);
    x->sur_w1t = a.take<__bf16>(192 * 128);
    x->sur_w2t = a.take<__bf16>(128 * 128);
    x->sur_phi = a.take<float>(B * 192);
    x->sur_z1 = a.take<float>(B * 128);
    x->sur_h1 = a.take<float>(B * 128);
    x->sur_z2 = a.take<float>(B * 128);
    x->sur_h2 = a.take<float>(B * 128);
    x->sur_out = a.take<float>(B);
    x->sur_dout = a.take<float>(B);
    x->sur_lterm = a.take<double>(B);
    x->sur_pred = a.take<float>(z.cand_cap);
    x->sur_flag = a.take<uint8_t>(z.cand_cap);
    x->sur_hist = a.take<uint32_t>(4096);
    x->sur_thr = a.take<uint32_t>(64);
    x->sur_cnt = a.take<int64_t>(16);
    x->sur_ri = a.take<int32_t>(2 * B);
    x->sur_rj = a.take<int32_t>(2 * B);
    x->sur_ry = a.take<float>(2 * B);
  }
  if (c->model == REC_GAUSS) {
    x->sc_kp = (int)((2 * c->M + 31) / 32 * 32);
    x->sc_a = a.take<__bf16>(N * x->sc_kp);
    x->sc_b = a.take<__bf16>(N * x->sc_kp);
    x->sc_nrm = a.take<float>(N);
    x->sc_th2 = a.take<float>(N);
    x->sc_sq = a.take<float>(N);
    x->sc_hist = a.take<uint32_t>(4096);
    x->sc_tau = a.take<float>(64);
  } else {
    x->sc_l1 = a.take<float>(N);
    x->sc_cv = a.take<float>(N);
    x->sc_wa = a.take<float>(z.max_nnz);
    x->sc_hist = a.take<uint32_t>(4096);
    x->sc_tau = a.take<float>(64);
  }
}

__global__ void k_check_pairs(const int32_t* I, const int32_t* J, int64_t P, int64_t N, int32_t* err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int i = I[p], j = J[p];
  if (i < 0 || j < 0 || i >= N || j >= N || i == j) atomicOr(err, 1);
}

// S strictly increasing and inside [0, N)
__global__ void k_check_set(const int32_t* S, int64_t n, int64_t N, int32_t* err) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  if (S[a] < 0 || S[a] >= N || (a > 0 && S[a - 1] >= S[a])) atomicOr(err, 1);
}

template <class R>
__global__ void k_fields_out(const R* H, int64_t N, int64_t M, int64_t Mp, double* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * M) return;
  int64_t i = e / M, s = e % M;
  out[e] = (double)H[i * Mp + s];
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

rec_status fail(rec_ctx* ctx, rec_status s, const char* msg) {
  if (ctx && msg) ctx->err = msg;
  return s;
}

rec_status read_err(rec_ctx* ctx, int32_t* e) {
  REC_HIP(hipMemcpyAsync(e, ctx->err_flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  return REC_OK;
}

rec_status clear_err(rec_ctx* ctx) {
  REC_HIP(hipMemsetAsync(ctx->err_flag, 0, 4, ctx->stream));
  return REC_OK;
}

#define REC_TRY(expr)                       \
  do {                                      \
    rec_status s_ = (expr);                 \
    if (s_ != REC_OK) return s_;            \
  } while (0)

#define REC_CHECK_CTX(ctx)                                                    \
  do {                                                                        \
    if (!(ctx)) return REC_E_INVAL;                                           \
    if ((ctx)->state != REC_OK) return fail(ctx, REC_E_STATE, "context poisoned by an earlier failure; call rec_set_model"); \
  } while (0)

}  // namespace

// Sum of the work-counter copies (synchronises).
rec_status rec_work_read(rec_ctx* ctx, int64_t out[8]) {
  std::vector<int64_t> h(REC_WORK_N * REC_WORK_COPIES);
  REC_HIP(hipMemcpyAsync(h.data(), ctx->work, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  for (int q = 0; q < REC_WORK_N; ++q) out[q] = 0;
  for (int c = 0; c < REC_WORK_COPIES; ++c)
    for (int q = 0; q < REC_WORK_N; ++q) out[q] += h[REC_WORK_N * c + q];
  return REC_OK;
}

namespace {

// refresh fields from W with the current theta, refit theta, evaluate
rec_status refresh(rec_ctx* ctx, double* obj) {
  REC_TRY(rec_rebuild_fields_fit_theta(ctx));
  return rec_eval_objective(ctx, obj);
}

}  // namespace

extern "C" {

const char* rec_status_str(rec_status s) {
  switch (s) {
    case REC_OK: return "ok";
    case REC_E_INVAL: return "invalid argument";
    case REC_E_NOMEM: return "workspace too small";
    case REC_E_HIP: return "HIP runtime error";
    case REC_E_NUMERIC: return "numeric error";
    case REC_E_STATE: return "context in failed state";
  }
  return "unknown status";
}

const char* rec_last_error(const rec_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

rec_status rec_workspace_size(const rec_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return REC_E_INVAL;
  Sizes z;
  const char* why = nullptr;
  rec_status s = plan(cfg, &z, &why);
  if (s != REC_OK) return s;
  rec_ctx tmp;
  tmp.cfg = *cfg;
  Arena a;
  a.base = nullptr;
  a.size = 0;
  layout(&tmp, cfg, z, a);
  *bytes = a.used + 256;
  return REC_OK;
}

// ---- static scratch of rec_score_pairs_noalloc ----
// Layout: [0, 8) the kink screen's queue counter, [8, 24) error flags,
// [256, 256 + 4 REC_NOALLOC_MAX_PAIRS) the queue (one 32-bit entry per pair).
// Each device holds its own copy for the life of the process.
constexpr int64_t REC_NOALLOC_MAX_PAIRS = int64_t(1) << 20;
constexpr size_t REC_NOALLOC_BYTES = 256 + 4 * (size_t)REC_NOALLOC_MAX_PAIRS;
static __device__ __align__(256) unsigned char scratch[REC_NOALLOC_BYTES];

namespace {
constexpr int REC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[REC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device (the host-side name is not a device address).
rec_status scratch_for_current_device(int dev, void** out) {
  if (dev < 0 || dev >= REC_MAX_DEVICES) return REC_E_INVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return REC_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return REC_OK;
}

__global__ void k_zero_scratch_head(int64_t* p) {
  if (threadIdx.x < 3) p[threadIdx.x] = 0;   // counter and the 16 bytes of error flags
}
}  // namespace

rec_status rec_create(const rec_config* cfg, const void* X_dev, void* ws_dev, size_t ws_bytes,
                      void* stream, rec_ctx** out) {
  if (!cfg || !X_dev || !ws_dev || !out) return REC_E_INVAL;
  *out = nullptr;
  Sizes z;
  const char* why = nullptr;
  rec_status s = plan(cfg, &z, &why);
  if (s != REC_OK) return s;
  rec_ctx* ctx = new (std::nothrow) rec_ctx();
  if (!ctx) return REC_E_NOMEM;
  ctx->cfg = *cfg;
  if (ctx->cfg.nnd_eps <= 0) ctx->cfg.nnd_eps = 1e-3;
  ctx->stream = (hipStream_t)stream;
  ctx->fp32 = cfg->prec == REC_FP32;
  ctx->m_default = z.m;
  // the update dataflow's bound on one wait (polls of a predecessor's flag);
  // REC_FLOW_SPIN_LIMIT overrides it (0: a pair that must wait ends the
  // launch with an error, the way the failure path is exercised)
  if (const char* e = std::getenv("REC_FLOW_SPIN_LIMIT")) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end != e && v >= 0) ctx->flow_spin_limit = v;
  }
  if (hipGetDevice(&ctx->dev) != hipSuccess) { delete ctx; return REC_E_HIP; }
  if (scratch_for_current_device(ctx->dev, &ctx->noalloc_scratch) != REC_OK) {
    delete ctx;
    return REC_E_HIP;
  }
  Arena a;
  a.base = (char*)(((uintptr_t)ws_dev + 255) & ~uintptr_t(255));
  a.size = ws_bytes - (size_t)(a.base - (char*)ws_dev);
  layout(ctx, cfg, z, a);
  if (a.used > a.size) { delete ctx; return REC_E_NOMEM; }
  Fields& F = ctx->F;
  F.N = cfg->N;
  F.M = cfg->M;
  F.Mp = z.Mp;
  F.npl = z.npl;
  F.model = cfg->model;
  // The kink screens compare sums of int8 copies with lambda.  Each copy
  // q = round(63.5 (y - tanh h)) (of the float-rounded value) is off by at
  // most 1/127 + 2^-22 a term (rec_q8), so a one-sided sum over M samples is
  // off the exact residual sum by M (1/127 + 2^-22), two sides by twice that;
  // the sums themselves are exact integers and their scaling rounds once
  // (2^-24 of a value below 2 M, in the 1e-6 lambda term).  The exact path
  // forms the same sums from working-precision values with float partial
  // sums of at most 32 terms per lane: M 2^-22 + 0.02 covers its rounding
  // (<= 64 lanes x 2 x 32 x 32 x 2^-24 < 4e-3).  A screened sum at most the
  // threshold therefore proves that the exact path finds |Phi(0)| <= lambda.
  const double eps_exact = (double)cfg->M * std::ldexp(1.0, -22) + 0.02 + 1e-6 * cfg->lambda;
  const double side = (double)cfg->M * (1.0 / 127.0 + std::ldexp(1.0, -22));
  F.scr = (float)(cfg->lambda - (side + eps_exact));
  F.scr2 = (float)(cfg->lambda - (2.0 * side + eps_exact));
  // The 4-bit copies u = round(7.5 (1 - y tanh h)) of 1 - y tanh h in [0, 2]
  // (computed in float from the working-precision tanh) are off by at most
  // 1/15 + 2^-20 a term, so with the signs exact a one-sided sum is off by
  // M (1/15 + 2^-20).  The kink kernel forms S = 7.5 x (the screened sum) in
  // exact integers, so |S| <= floor(7.5 (lambda - bound - eps_exact)) proves
  // |Phi(0)| <= lambda; a pair that fails goes on to the int8 test.
  const double side4 = (double)cfg->M * (1.0 / 15.0 + std::ldexp(1.0, -20));
  auto t4of = [](double v) { return (int32_t)std::min(2147483647.0, std::max(-1.0, std::floor(7.5 * v))); };
  F.t4 = t4of(cfg->lambda - (side4 + eps_exact));
  F.t42 = t4of(cfg->lambda - (2.0 * side4 + eps_exact));
  auto bad = [&](rec_status st) { delete ctx; return st; };
  if (hipMemsetAsync(ctx->err_flag, 0, 16, ctx->stream) != hipSuccess) return bad(REC_E_HIP);
  if (hipMemsetAsync(ctx->counter, 0, 16 * 8, ctx->stream) != hipSuccess) return bad(REC_E_HIP);
  if (hipMemsetAsync(ctx->work, 0, REC_WORK_N * 8 * REC_WORK_COPIES, ctx->stream) != hipSuccess) return bad(REC_E_HIP);
  rec_wtable_clear(ctx);
  if (rec_load_data(ctx, X_dev, cfg->ldx) != REC_OK) return bad(REC_E_HIP);
  hipLaunchKernelGGL(k_fill_f64, dim3((cfg->N + 255) / 256), dim3(256), 0, ctx->stream, F.theta,
                     cfg->N, cfg->model == REC_GAUSS ? 1.0 : 0.0);
  int32_t e = 0;
  if (read_err(ctx, &e) != REC_OK) return bad(REC_E_HIP);
  if (e & 4) return bad(REC_E_NUMERIC);
  double obj;
  if (refresh(ctx, &obj) != REC_OK) return bad(REC_E_HIP);
  if (rec_sur_init(ctx) != REC_OK) return bad(REC_E_HIP);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bad(REC_E_HIP);
  *out = ctx;
  return REC_OK;
}

rec_status rec_destroy(rec_ctx* ctx) {
  if (!ctx) return REC_E_INVAL;
  hipStreamSynchronize(ctx->stream);
  delete ctx;
  return REC_OK;
}

rec_status rec_score_pairs(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                           double* gain_dev, double* wopt_dev) {
  REC_CHECK_CTX(ctx);
  if (P < 0 || (P > 0 && (!i_dev || !j_dev || !gain_dev))) return fail(ctx, REC_E_INVAL, "bad arguments");
  if (P == 0) return REC_OK;
  REC_TRY(clear_err(ctx));
  REC_TRY(rec_launch_score(ctx, P, i_dev, j_dev, nullptr, gain_dev, wopt_dev, nullptr));
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 1) return fail(ctx, REC_E_INVAL, "pair index out of range or i == j");
  return REC_OK;
}

rec_status rec_score_pairs_noalloc(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                                   double* gain_dev, double* wopt_dev) {
  REC_CHECK_CTX(ctx);
  if (P < 0 || (P > 0 && (!i_dev || !j_dev || !gain_dev))) return fail(ctx, REC_E_INVAL, "bad arguments");
  if (P > REC_NOALLOC_MAX_PAIRS)
    return fail(ctx, REC_E_INVAL, "P exceeds the static scratch of rec_score_pairs_noalloc (2^20 pairs per call)");
  if (P == 0) return REC_OK;
  char* base = static_cast<char*>(ctx->noalloc_scratch);
  if (!base) return fail(ctx, REC_E_STATE, "static scratch not set up for this device");
  int64_t* head = reinterpret_cast<int64_t*>(base);
  int32_t* err = reinterpret_cast<int32_t*>(base + 8);
  hipLaunchKernelGGL(k_zero_scratch_head, dim3(1), dim3(64), 0, ctx->stream, head);
  const ScoreScratch ss{reinterpret_cast<uint32_t*>(base + 256), head, REC_NOALLOC_MAX_PAIRS, err,
                        nullptr, true};
  REC_TRY(rec_launch_score_with(ctx, P, i_dev, j_dev, gain_dev, wopt_dev, ss));
  REC_HIP(hipGetLastError());
  int32_t e = 0;
  REC_HIP(hipMemcpyAsync(&e, err, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  if (e & 1) return fail(ctx, REC_E_INVAL, "pair index out of range or i == j");
  if (e & 512) return fail(ctx, REC_E_HIP, "static queue overflow");
  return REC_OK;
}

rec_status rec_grad_pairs(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                          double* dist_dev) {
  REC_CHECK_CTX(ctx);
  if (P < 0 || (P > 0 && (!i_dev || !j_dev || !dist_dev))) return fail(ctx, REC_E_INVAL, "bad arguments");
  if (P == 0) return REC_OK;
  REC_TRY(clear_err(ctx));
  ctx->grad_dist = true;
  rec_status st = rec_launch_score(ctx, P, i_dev, j_dev, nullptr, dist_dev, nullptr, nullptr);
  ctx->grad_dist = false;
  REC_TRY(st);
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 1) return fail(ctx, REC_E_INVAL, "pair index out of range or i == j");
  return REC_OK;
}

rec_status rec_find_best_candidates(rec_ctx* ctx, int64_t m, int32_t search, int32_t* i_dev, int32_t* j_dev,
                         double* gain_dev, int64_t* n_out_host, rec_sweep_stats* st) {
  REC_CHECK_CTX(ctx);
  if (m < 1 || !i_dev || !j_dev || !gain_dev || !n_out_host || search < 0 || search > REC_SEARCH_GRADIENT)
    return fail(ctx, REC_E_INVAL, "bad arguments");
  if (m > ctx->best_cap) return fail(ctx, REC_E_INVAL, "m exceeds the capacity planned for kappa");
  REC_TRY(clear_err(ctx));
  rec_sweep_stats local{};
  double t0 = now_ms();
  int64_t n = 0;
  rec_status s = rec_search_best(ctx, m, search, &n, &local);
  if (s != REC_OK) return s;
  REC_HIP(hipMemcpyAsync(i_dev, ctx->best_i, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  REC_HIP(hipMemcpyAsync(j_dev, ctx->best_j, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  REC_HIP(hipMemcpyAsync(gain_dev, ctx->best_g, n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  *n_out_host = n;
  local.n_best = n;
  local.t_search_ms = now_ms() - t0;
  if (st) *st = local;
  return REC_OK;
}

rec_status rec_apply_updates(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                             double* delta_host) {
  REC_CHECK_CTX(ctx);
  if (P < 0 || (P > 0 && (!i_dev || !j_dev))) return fail(ctx, REC_E_INVAL, "bad arguments");
  if (P > ctx->best_cap) return fail(ctx, REC_E_INVAL, "too many pairs for one call");
  double d = 0.0;
  if (P > 0) {
    REC_TRY(clear_err(ctx));
    hipLaunchKernelGGL(k_check_pairs, dim3((P + 255) / 256), dim3(256), 0, ctx->stream, i_dev, j_dev,
                       P, ctx->cfg.N, ctx->err_flag);
    int32_t e = 0;
    REC_TRY(read_err(ctx, &e));
    if (e & 1) return fail(ctx, REC_E_INVAL, "pair index out of range or i == j");
    REC_HIP(hipMemcpyAsync(ctx->best_i, i_dev, P * 4, hipMemcpyDeviceToDevice, ctx->stream));
    REC_HIP(hipMemcpyAsync(ctx->best_j, j_dev, P * 4, hipMemcpyDeviceToDevice, ctx->stream));
    int64_t acc, rounds;
    rec_status s = rec_apply_best(ctx, P, ctx->best_i, ctx->best_j, &d, &acc, &rounds);
    if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  }
  if (delta_host) *delta_host = d;
  return REC_OK;
}

rec_status rec_gcd_sweep(rec_ctx* ctx, int32_t search, rec_sweep_stats* st) {
  REC_CHECK_CTX(ctx);
  if (search < 0 || search > REC_SEARCH_GRADIENT) return fail(ctx, REC_E_INVAL, "unknown search");
  REC_TRY(clear_err(ctx));
  rec_sweep_stats S{};
  double t0 = now_ms();
  int64_t n = 0;
  rec_status s = rec_search_best(ctx, ctx->m_default, search, &n, &S);
  if (s != REC_OK) return s;
  // E_best keeps the positive gains of the best m: a pair of zero gain would
  // leave W as it is, and the ties among zero gains are not chosen at all.
  // Under the gradient distance the ranking is not by gain: every pair stays.
  if (search != REC_SEARCH_GRADIENT && search != REC_SEARCH_SCREEN)
    REC_TRY(rec_positive_prefix(ctx, ctx->best_g, n, &n));
  double t1 = now_ms();
  int64_t acc = 0, rounds = 0;
  double delta = 0.0;
  s = rec_apply_best(ctx, n, ctx->best_i, ctx->best_j, &delta, &acc, &rounds);
  if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  double t2 = now_ms();
  double obj = 0.0;
  s = refresh(ctx, &obj);
  if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  double t3 = now_ms();
  S.objective = obj;
  S.delta = delta;
  S.accepted = acc;
  S.n_best = n;
  S.rounds = rounds;
  S.t_search_ms = t1 - t0;
  S.t_update_ms = t2 - t1;
  S.t_theta_ms = t3 - t2;
  if (st) *st = S;
  return REC_OK;
}

rec_status rec_cd_sweep(rec_ctx* ctx, rec_sweep_stats* st) {
  REC_CHECK_CTX(ctx);
  REC_TRY(clear_err(ctx));
  const int64_t N = ctx->cfg.N, n = N + (N & 1);
  double t0 = now_ms();
  REC_HIP(hipMemsetAsync(ctx->cd_acc, 0, sizeof(double) * (n / 2), ctx->stream));
  int64_t* changes = ctx->counter + 6;
  REC_HIP(hipMemsetAsync(changes, 0, sizeof(int64_t), ctx->stream));
  ++ctx->w_version;   // the rounds write W
  ctx->w_any = true;
  for (int64_t r = 0; r + 1 < n; ++r) {
    rec_status s = rec_launch_cd_round(ctx, r, n, ctx->cd_acc, changes);
    if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  }
  REC_TRY(rec_sum_device(ctx, ctx->cd_acc, n / 2, ctx->dresult + 3));
  double delta = 0.0;
  int64_t acc = 0;
  REC_HIP(hipMemcpyAsync(&delta, ctx->dresult + 3, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipMemcpyAsync(&acc, changes, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 2) { ctx->state = REC_E_STATE; return fail(ctx, REC_E_NOMEM, "W table full"); }
  double t1 = now_ms();
  double obj = 0.0;
  rec_status s = refresh(ctx, &obj);
  if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  double t2 = now_ms();
  if (st) {
    rec_sweep_stats S{};
    S.objective = obj;
    S.delta = delta;
    S.accepted = acc;
    S.n_best = ctx->cfg.model == REC_KINETIC ? N * (N - 1) : N * (N - 1) / 2;
    S.pair_evals = S.n_best;
    S.rounds = n - 1;
    S.t_update_ms = t1 - t0;
    S.t_theta_ms = t2 - t1;
    *st = S;
  }
  return REC_OK;
}

rec_status rec_search_levels(rec_ctx* ctx, int32_t cap, int64_t* level_n_host, int32_t* levels_host) {
  if (!ctx || !levels_host || cap < 0 || (cap > 0 && !level_n_host)) return REC_E_INVAL;
  *levels_host = ctx->last_levels;
  for (int l = 0; l < ctx->last_levels && l < cap; ++l) level_n_host[l] = ctx->last_level_n[l];
  return REC_OK;
}

rec_status rec_theta_update(rec_ctx* ctx, double* objective_host) {
  REC_CHECK_CTX(ctx);
  double obj;
  rec_status s = refresh(ctx, &obj);
  if (s != REC_OK) { ctx->state = REC_E_STATE; return s; }
  if (objective_host) *objective_host = obj;
  return REC_OK;
}

rec_status rec_objective(rec_ctx* ctx, double* objective_host) {
  REC_CHECK_CTX(ctx);
  if (!objective_host) return fail(ctx, REC_E_INVAL, "null output");
  return rec_eval_objective(ctx, objective_host);
}

rec_status rec_get_model(rec_ctx* ctx, int64_t cap, int32_t* ei_dev, int32_t* ej_dev, double* w_dev,
                         double* theta_dev, int64_t* nnz_host) {
  if (!ctx || !nnz_host || cap < 0) return REC_E_INVAL;
  if (cap > 0 && (!ei_dev || !ej_dev || !w_dev)) return fail(ctx, REC_E_INVAL, "null output");
  int64_t nnz = 0;
  REC_TRY(rec_wtable_compact(ctx, &nnz));
  int64_t c = std::min(cap, nnz);
  if (c > 0) {
    REC_HIP(hipMemcpyAsync(ei_dev, ctx->wi, c * 4, hipMemcpyDeviceToDevice, ctx->stream));
    REC_HIP(hipMemcpyAsync(ej_dev, ctx->wj, c * 4, hipMemcpyDeviceToDevice, ctx->stream));
    REC_HIP(hipMemcpyAsync(w_dev, ctx->wv, c * 8, hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (theta_dev)
    REC_HIP(hipMemcpyAsync(theta_dev, ctx->F.theta, ctx->cfg.N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  *nnz_host = nnz;
  return REC_OK;
}

rec_status rec_set_model(rec_ctx* ctx, int64_t nnz, const int32_t* ei_dev, const int32_t* ej_dev,
                         const double* w_dev, const double* theta_dev) {
  if (!ctx || nnz < 0 || (nnz > 0 && (!ei_dev || !ej_dev || !w_dev))) return REC_E_INVAL;
  if (nnz > ctx->max_nnz) return fail(ctx, REC_E_NOMEM, "more entries than max_nnz");
  REC_TRY(clear_err(ctx));
  rec_wtable_clear(ctx);
  REC_TRY(rec_wtable_insert_list(ctx, nnz, ei_dev, ej_dev, w_dev));
  if (theta_dev)
    REC_HIP(hipMemcpyAsync(ctx->F.theta, theta_dev, ctx->cfg.N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 8) { ctx->state = REC_E_STATE; return fail(ctx, REC_E_INVAL, "bad W entry (index or value)"); }
  if (e & 2) { ctx->state = REC_E_STATE; return fail(ctx, REC_E_NOMEM, "W table full"); }
  REC_TRY(rec_rebuild_fields(ctx));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  ctx->state = REC_OK;
  return REC_OK;
}

rec_status rec_get_fields(rec_ctx* ctx, double* H_dev) {
  if (!ctx || !H_dev) return REC_E_INVAL;
  int64_t n = ctx->cfg.N * ctx->cfg.M;
  if (ctx->fp32)
    hipLaunchKernelGGL(k_fields_out<float>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       (const float*)ctx->F.H, ctx->cfg.N, ctx->cfg.M, ctx->F.Mp, H_dev);
  else
    hipLaunchKernelGGL(k_fields_out<double>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       (const double*)ctx->F.H, ctx->cfg.N, ctx->cfg.M, ctx->F.Mp, H_dev);
  REC_HIP(hipStreamSynchronize(ctx->stream));
  return REC_OK;
}

rec_status rec_knn(rec_ctx* ctx, int64_t n, const int32_t* S_dev, int32_t k, int32_t level,
                   int32_t mode, int32_t* nbr_dev, double* gain_dev, int32_t* iters_host) {
  REC_CHECK_CTX(ctx);
  if (n < 2 || n > ctx->cfg.N || k < 1 || k > n - 1 || !S_dev || !nbr_dev || !gain_dev ||
      (mode != REC_SEARCH_NNDESCENT && mode != REC_SEARCH_EXACT_KNN && mode != REC_SEARCH_GRADIENT))
    return fail(ctx, REC_E_INVAL, "bad arguments");
  REC_TRY(clear_err(ctx));
  hipLaunchKernelGGL(k_check_set, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, S_dev, n,
                     ctx->cfg.N, ctx->err_flag);
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 1) return fail(ctx, REC_E_INVAL, "S must be strictly increasing node indices in [0, N)");
  int it = 0;
  ctx->grad_dist = mode == REC_SEARCH_GRADIENT;   // NNDescent under the gradient distance
  rec_status s = rec_search_knn(ctx, n, S_dev, k, level, mode == REC_SEARCH_EXACT_KNN ? 1 : 0,
                                nbr_dev, gain_dev, &it);
  ctx->grad_dist = false;
  if (s != REC_OK) return s;
  REC_HIP(hipStreamSynchronize(ctx->stream));
  if (iters_host) *iters_host = it;
  return REC_OK;
}

// ---- learned proposal ----
rec_status rec_sketch(rec_ctx* ctx, float* S_dev) {
  REC_CHECK_CTX(ctx);
  REC_TRY(rec_sur_sketch(ctx));
  if (S_dev)
    REC_HIP(hipMemcpyAsync(S_dev, ctx->sur_S, ctx->cfg.N * REC_SUR_SDIM * sizeof(float),
                           hipMemcpyDeviceToDevice, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  return REC_OK;
}

rec_status rec_mlp_params(rec_ctx* ctx, float* get_dev, const float* set_dev) {
  REC_CHECK_CTX(ctx);
  const size_t bytes = REC_SUR_NPARAM * sizeof(float);
  if (get_dev) REC_HIP(hipMemcpyAsync(get_dev, ctx->sur_par, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (set_dev) {
    REC_HIP(hipMemcpyAsync(ctx->sur_par, set_dev, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    REC_HIP(hipMemsetAsync(ctx->sur_m, 0, bytes, ctx->stream));
    REC_HIP(hipMemsetAsync(ctx->sur_v, 0, bytes, ctx->stream));
    ctx->sur_t = 0;
    REC_TRY(rec_sur_pack(ctx));
  }
  REC_HIP(hipStreamSynchronize(ctx->stream));
  return REC_OK;
}

namespace {
rec_status check_pairs_arg(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J) {
  REC_TRY(clear_err(ctx));
  hipLaunchKernelGGL(k_check_pairs, dim3((P + 255) / 256), dim3(256), 0, ctx->stream, I, J, P,
                     ctx->cfg.N, ctx->err_flag);
  int32_t e = 0;
  REC_TRY(read_err(ctx, &e));
  if (e & 1) return fail(ctx, REC_E_INVAL, "pair indices outside [0, N) or i == j");
  return REC_OK;
}
}  // namespace

rec_status rec_mlp_infer(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                         float* out_dev) {
  REC_CHECK_CTX(ctx);
  if (P < 0 || (P > 0 && (!i_dev || !j_dev || !out_dev))) return fail(ctx, REC_E_INVAL, "bad arguments");
  if (P == 0) return REC_OK;
  REC_TRY(check_pairs_arg(ctx, P, i_dev, j_dev));
  REC_TRY(rec_sur_infer(ctx, P, i_dev, j_dev, nullptr, nullptr, out_dev));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  return REC_OK;
}

rec_status rec_mlp_grad(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                        const float* y_dev, float* grad_dev, double* loss_host) {
  REC_CHECK_CTX(ctx);
  if (P < 1 || P > REC_SUR_BATCH || !i_dev || !j_dev || !y_dev)
    return fail(ctx, REC_E_INVAL, "bad arguments (1 <= P <= 8192)");
  REC_TRY(check_pairs_arg(ctx, P, i_dev, j_dev));
  REC_TRY(rec_sur_grad(ctx, P, i_dev, j_dev, y_dev));
  if (grad_dev)
    REC_HIP(hipMemcpyAsync(grad_dev, ctx->sur_g, REC_SUR_NPARAM * sizeof(float), hipMemcpyDeviceToDevice,
                           ctx->stream));
  double l = 0.0;
  REC_HIP(hipMemcpyAsync(&l, ctx->dresult + 8, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  if (loss_host) *loss_host = l;
  return REC_OK;
}

rec_status rec_mlp_train(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                         const float* y_dev, int32_t steps, float lr, double* loss_host) {
  REC_CHECK_CTX(ctx);
  if (P < 1 || P > REC_SUR_BATCH || !i_dev || !j_dev || !y_dev || steps < 1 || !(lr > 0.f))
    return fail(ctx, REC_E_INVAL, "bad arguments (1 <= P <= 8192, steps >= 1, lr > 0)");
  REC_TRY(check_pairs_arg(ctx, P, i_dev, j_dev));
  for (int s = 0; s < steps; ++s) {
    REC_TRY(rec_sur_grad(ctx, P, i_dev, j_dev, y_dev));
    REC_TRY(rec_sur_adam(ctx, lr));
  }
  REC_TRY(rec_sur_pack(ctx));
  double l = 0.0;
  REC_HIP(hipMemcpyAsync(&l, ctx->dresult + 8, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  if (loss_host) *loss_host = l;
  return REC_OK;
}

rec_status rec_surrogate_config(rec_ctx* ctx, double rho, double recall_min, int32_t train_steps,
                                float lr, int32_t audit_log2, int32_t zero_log2) {
  REC_CHECK_CTX(ctx);
  if (!(rho > 0.0 && rho <= 1.0) || !(recall_min >= 0.0 && recall_min <= 1.0) || train_steps < 0 ||
      !(lr > 0.f) || audit_log2 < 0 || audit_log2 > 20 || zero_log2 < 0 || zero_log2 > 30)
    return fail(ctx, REC_E_INVAL, "bad surrogate configuration");
  ctx->sur_rho = rho;
  ctx->sur_recall_min = recall_min;
  ctx->sur_steps = train_steps;
  ctx->sur_lr = lr;
  ctx->sur_audit = 1u << audit_log2;
  ctx->sur_zbits = zero_log2;
  return REC_OK;
}

rec_status rec_surrogate_stats(rec_ctx* ctx, double* out_host) {
  if (!ctx || !out_host) return REC_E_INVAL;
  for (int q = 0; q < 10; ++q) out_host[q] = ctx->sur_stats[q];
  return REC_OK;
}

rec_status rec_set_timing(rec_ctx* ctx, int32_t on) {
  if (!ctx) return REC_E_INVAL;
  REC_TRY(rec_timing_resolve(ctx));
  REC_TRY(rec_screen_resolve(ctx));
  for (int q = 0; q < 9; ++q) ctx->sc_stat[q] = 0.0;
  ctx->timing = on != 0;
  ctx->score_ms = 0.0;
  ctx->score_launches = ctx->score_pairs = 0;
  return rec_work_read(ctx, ctx->work_base);
}

rec_status rec_screen_time(rec_ctx* ctx, double* out_host) {
  if (!ctx || !out_host) return REC_E_INVAL;
  REC_TRY(rec_screen_resolve(ctx));
  for (int q = 0; q < 9; ++q) {
    out_host[q] = ctx->sc_stat[q];
    ctx->sc_stat[q] = 0.0;
  }
  return REC_OK;
}

rec_status rec_kernel_time(rec_ctx* ctx, double* score_ms_host, int64_t* launches_host,
                           int64_t* work_host) {
  if (!ctx) return REC_E_INVAL;
  REC_TRY(rec_timing_resolve(ctx));
  int64_t w[REC_WORK_N];
  REC_TRY(rec_work_read(ctx, w));
  if (score_ms_host) *score_ms_host = ctx->score_ms;
  if (launches_host) *launches_host = ctx->score_launches;
  if (work_host)
    for (int q = 0; q < REC_WORK_N; ++q) work_host[q] = w[q] - ctx->work_base[q];
  for (int q = 0; q < REC_WORK_N; ++q) ctx->work_base[q] = w[q];
  ctx->score_ms = 0.0;
  ctx->score_launches = ctx->score_pairs = 0;
  return REC_OK;
}

}  // extern "C"
