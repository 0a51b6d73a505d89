// Context state of the library and the host-side entry points of each
// kernel family (definitions in the .hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/rec.h"
#include "common.hpp"

constexpr int64_t REC_TAIL_ROWS = 256;   // zero rows after the N rows of xs and rq

// Device view of the data and fields, passed by value to kernels.
struct Fields {
  const int8_t* xs;     // N x Mp input side +-1 (kinetic: x_{j,t-1}); padding 0
  const int8_t* ys;     // N x Mp target side (kinetic: x_{i,t}); symmetric: == xs
  const float* xf;      // Gaussian data N x Mp (padding 0), else null
  void* H;              // N x Mp fields (Gaussian: residuals), real
  void* T;              // N x Mp tanh(H) (Ising/kinetic), real
  const double* sq;     // Gaussian: ||x_i||^2
  double* theta;        // N
  // Ising / kinetic screen data.  xq, yq: N x 64 lane words of npl bits
  // (16-bit words when npl <= 16, else 32-bit: rec_sign_word), bit c*VEC + k
  // of lane l is sample c*64*VEC + l*VEC + k of xs (yq: ys) being +1 (padding
  // reads as -1 and is cancelled by zeros on the other side); rq: N x Mp
  // int8 residuals q = round(63.5 (y - tanh h)) (padding 0).  rq and xs
  // carry REC_TAIL_ROWS zero rows past N (the contraction's tiles never need
  // a bound check).
  // u4: N x (rec_u4_words(npl) x 64) lane words, nibble n = c*VEC + k of
  // lane l (word n / 8, bits 4 (n % 8)) holding round(7.5 (1 - y tanh h)) of
  // sample c*64*VEC + l*VEC + k (0 in the padding): with the sign of y from
  // the sign rows, y - tanh h = y (1 - y tanh h), 1 - y tanh h in [0, 2].
  const void* xq;
  const void* yq;
  int8_t* rq;
  uint32_t* u4;
  float scr;            // kink screen, one int8 side: lambda minus its error bound and the exact path's rounding
  float scr2;           // kink screen, two int8 sides (Ising): the same with both sides' bounds
  int32_t t4;           // kink screen, one 4-bit side: integer sums |S| <= t4 prove |Phi(0)| <= lambda
  int32_t t42;          // kink screen, two 4-bit sides (Ising)
  int64_t N, M, Mp;     // valid samples M, padded row length Mp = 64 * npl
  int npl;              // samples per lane
  int model;            // rec_model
};

// lane word of the sign rows xq / yq: npl bits per lane, stored in 16 bits
// when they fit (the row is then 128 bytes), else 32
template <int NPL>
using rec_sign_t = typename std::conditional<(NPL <= 16), uint16_t, uint32_t>::type;
template <int NPL>
__device__ __forceinline__ uint32_t rec_sign_word(const void* q, int64_t row, int lane) {
  return (uint32_t)reinterpret_cast<const rec_sign_t<NPL>*>(q)[row * REC_WAVE + lane];
}

// 4-bit residual rows: lane words per row and the nibble of one sample
__host__ __device__ constexpr int rec_u4_words(int npl) { return npl < 8 ? 1 : npl / 8; }
__device__ __forceinline__ uint32_t rec_u4(float u) {   // u = 1 - y tanh h in [0, 2]
  return (uint32_t)fminf(fmaxf(rintf(u * 7.5f), 0.f), 15.f);
}
// bits b_0..b_7 of a byte spread to the nibbles of a word (nibble k = b_k)
__device__ __forceinline__ uint32_t rec_spread8(uint32_t b) {
  b = (b | (b << 12)) & 0x000F000Fu;
  b = (b | (b << 6)) & 0x03030303u;
  return (b | (b << 3)) & 0x11111111u;
}

// Open-addressing table of W entries: key = pair key, value = weight.
struct WTable {
  uint64_t* keys;
  double* vals;
  uint64_t mask;        // capacity - 1
  uint32_t* bloom;      // REC_WBLOOM_WORDS words: a filter of the keys ever inserted
};

// The key filter of W: each inserted key sets two bits of one 32-bit word
// (a blocked Bloom filter, 256 KB, resident in L2).  A key whose bits are not
// both set was never inserted, and its lookup ends without a probe of the
// table (a random line of keys in HBM).  Keys are never removed, so the
// filter only grows until the table is cleared.
constexpr int REC_WBLOOM_WORDS = 1 << 16;
__device__ __forceinline__ void rec_wbloom_pos(uint64_t key, uint32_t* word, uint32_t* bits) {
  const uint64_t h = key * 0x9E3779B97F4A7C15ull;
  *word = (uint32_t)(h >> 48);
  *bits = (1u << ((h >> 5) & 31u)) | (1u << ((h >> 10) & 31u));
}
__device__ __forceinline__ void rec_wbloom_set(const WTable& W, uint64_t key) {
  uint32_t w, b;
  rec_wbloom_pos(key, &w, &b);
  atomicOr(W.bloom + w, b);
}
__device__ __forceinline__ bool rec_wbloom_maybe(const WTable& W, uint64_t key) {
  uint32_t w, b;
  rec_wbloom_pos(key, &w, &b);
  return (W.bloom[w] & b) == b;
}

// Score memo inside one FindBest call [App. B, caching].
struct Cache {
  uint64_t* keys;
  double* vals;
  uint64_t mask;
  double* ovf;          // values of pairs that found no free slot
  int64_t ovf_cap;
};

constexpr int REC_MAX_PROBE = 64;

struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  template <class T>
  T* take(size_t n) {
    size_t bytes = ((n * sizeof(T)) + 255) & ~size_t(255);
    size_t off = used;
    used += bytes;
    if (base == nullptr || used > size) return nullptr;
    return reinterpret_cast<T*>(base + off);
  }
};

struct SortBufs {
  uint64_t* khi[2];
  uint64_t* klo[2];
  uint32_t* val[2];
  uint32_t* hist;
  int64_t cap;
};

struct rec_ctx {
  rec_config cfg;
  hipStream_t stream;
  int dev;
  void* noalloc_scratch = nullptr;   // this device's address of the static scratch
  double* cd_acc = nullptr;          // CD sweep: |dW| per round-robin pair slot (N/2 + 1)
  int64_t last_level_n[64] = {};     // node count of each FindBest level of the last search
  int32_t last_levels = 0;
  rec_status state = REC_OK;
  std::string err;
  bool fp32;
  int64_t m_default;

  Fields F;
  WTable W;
  Cache C;
  SortBufs sb;
  int64_t max_nnz;
  // W changes bump w_version; a compaction (sorted lists, row lists) is
  // reused while the version it was made at is current
  uint64_t w_version = 1, w_compacted = 0;
  // false only between a clear of the W table and the next launch that may
  // insert into it: the scoring kernels then skip the lookups (each a random
  // cache line of keys) and take w = 0
  bool w_any = true;
  // bound on one wait of the update dataflow, in polls of a flag (about
  // 1-2 us each): far beyond any chain of predecessors, so hitting it means a
  // broken schedule, reported as an error instead of a hang
  int64_t flow_spin_limit = int64_t(1) << 24;
  int64_t w_nnz = 0;

  // W as sorted row lists (CSR) for the field rebuild
  int64_t* row_off;     // N+1
  int32_t* col;         // 2 max_nnz
  double* colw;         // 2 max_nnz
  // scratch for compaction of the W table
  int32_t* wi; int32_t* wj; double* wv;   // max_nnz each
  int64_t* counter;     // small device counters [16]
  int64_t* work;        // pair-score work counters, REC_WORK_N x REC_WORK_COPIES
  double* dscratch;     // per-block partial sums (N)
  double* dresult;      // small double results [16]
  int32_t* err_flag;    // device error flag

  // search state (see search.hip)
  int64_t list_cap;     // capacity of KNN list entries (>= 4m + N)
  int32_t *Gidx, *Gidx2; double *Ggain, *Ggain2;
  int32_t *S, *S2, *loc;
  int64_t *cnt, *off;   // per node counts / offsets (N + 1)
  int64_t cand_cap;
  int32_t* cand_v; int32_t* cand_gi; uint32_t* cand_slot;
  int32_t *ts_i, *ts_j; uint32_t* ts_slot;    // to-score list
  int64_t* inoff;       // N + 1
  int32_t* in_src;      // list_cap: capped in-neighbours, k per node
  int32_t* capcnt;      // N
  uint64_t* dset_keys; uint64_t dset_mask;
  uint64_t* pset_keys; uint64_t pset_mask;
  int64_t pool_cap;
  uint64_t *pool_hi, *pool_lo;
  int32_t* flags;       // N
  int64_t* scan_tmp;    // block sums for scans
  // E_best and update rounds
  int64_t best_cap;
  int32_t *best_i, *best_j; double* best_g;
  int32_t* pred;        // 2 best_cap: previous pair on each row of a pair being applied
  int32_t* pend[2];     // best_cap each: pending pairs of the update rounds (ping-pong)
  uint8_t* done;        // best_cap
  double* dw;           // best_cap
  int32_t* ready;       // best_cap: the pairs of the current update round
  int32_t* depth;       // best_cap: the round each applied pair ran in (1-based)
  int64_t* best_slot;   // best_cap: W table slot of each pair being applied
  // exhaustive search chunk buffers
  int64_t ex_cap;
  // queue of the screened scoring's unsettled pairs (k_kink -> k_exact)
  uint32_t* scr_queue = nullptr;
  int64_t scr_qcap = 0;
  // kinetic model inside FindBest: pairs are unordered and scored by the
  // larger of the two directed gains
  bool sym_search = false;
  // search distance: the exact gain, or (true) the absolute gradient
  bool grad_dist = false;
  // screening contraction, Gaussian: bf16 operands N x sc_kp, row norms,
  // theta^2, |x|^2; all models: histogram and threshold
  __bf16* sc_a = nullptr;
  __bf16* sc_b = nullptr;
  int sc_kp = 0;
  float *sc_nrm = nullptr, *sc_th2 = nullptr, *sc_sq = nullptr, *sc_tau = nullptr;
  // Ising / kinetic screen: per node |r_i|_1 and curvature sum (1 - t^2);
  // per current coupling its gradient from the int8 rows (max_nnz)
  float *sc_l1 = nullptr, *sc_cv = nullptr, *sc_wa = nullptr;
  // screen instrumentation: [0] full-pass ms, [1] full-pass launches, [2]
  // their algorithmic flops, [3] sample-pass ms, [4] sample launches, [5]
  // screen calls, [6] pairs decided, [7] pairs rescored exactly, [8] calls
  // that needed a second collect pass
  double sc_stat[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  struct ScrEv { hipEvent_t a, b; int kind; double flops; };
  std::vector<ScrEv> sev;
  size_t sev_used = 0;
  uint32_t* sc_hist = nullptr;
  // learned proposal (surrogate.hip): projection bits, sketches, parameters,
  // Adam state, bf16 weight copies, training work arrays
  uint32_t* sur_pbits = nullptr;
  float* sur_S = nullptr;
  __bf16* sur_Sb = nullptr;
  float *sur_par = nullptr, *sur_m = nullptr, *sur_v = nullptr, *sur_g = nullptr;
  __bf16 *sur_w1t = nullptr, *sur_w2t = nullptr;
  float *sur_phi = nullptr, *sur_z1 = nullptr, *sur_h1 = nullptr, *sur_z2 = nullptr, *sur_h2 = nullptr;
  float *sur_out = nullptr, *sur_dout = nullptr;
  double* sur_lterm = nullptr;
  int64_t sur_t = 0;
  // proposal inside the search: predictions, flags, threshold, counters, records
  float* sur_pred = nullptr;
  uint8_t* sur_flag = nullptr;
  uint32_t *sur_hist = nullptr, *sur_thr = nullptr;
  int64_t* sur_cnt = nullptr;
  int32_t *sur_ri = nullptr, *sur_rj = nullptr;
  float* sur_ry = nullptr;
  // configuration and state
  double sur_rho = 0.25, sur_recall_min = 0.99;
  int sur_steps = 50, sur_zbits = 6;
  uint32_t sur_audit = 16;
  float sur_lr = 1e-3f;
  int sur_mode = 0;            // inside a FindBest call: 0 off, 1 shadow (plain search), 2 active
  bool sur_trained = false;
  double sur_recall = -1.0;    // last estimate (-1: none yet)
  double sur_stats[10] = {0, -1, 0, 0, 0, 0, 0, 0, 0, 0};
  // pair-score kernel timing (instrumentation)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  double score_ms = 0.0;
  int64_t score_launches = 0, score_pairs = 0;
  int64_t work_base[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // work counters when timing was switched on
  ~rec_ctx() {
    for (auto& e : ev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : sev) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  }
};

rec_status rec_timing_resolve(rec_ctx* ctx);
rec_status rec_work_read(rec_ctx* ctx, int64_t out[8]);

// ---- launch helpers (implemented in the .hip files) ----
#define REC_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return REC_E_HIP;                                                        \
    }                                                                          \
  } while (0)

// fields.hip
rec_status rec_load_data(rec_ctx* ctx, const void* X, int64_t ldx);
rec_status rec_rebuild_fields(rec_ctx* ctx);              // from W table and theta
rec_status rec_fit_theta(rec_ctx* ctx);                   // theta update + field shift
rec_status rec_rebuild_fields_fit_theta(rec_ctx* ctx);    // both in one pass over the rows
rec_status rec_eval_objective(rec_ctx* ctx, double* out);
rec_status rec_wtable_compact(rec_ctx* ctx, int64_t* nnz); // W table -> wi/wj/wv (sorted)
void rec_wtable_clear(rec_ctx* ctx);
// sum of n doubles into *out (device), deterministic; uses dscratch
rec_status rec_sum_device(rec_ctx* ctx, const double* x, int64_t n, double* out);
rec_status rec_wtable_insert_list(rec_ctx* ctx, int64_t n, const int32_t* ei, const int32_t* ej,
                                  const double* w);

// score.hip
// Score pairs (I[p], J[p]); results to gain_out[slot ? slot[p] : p] (and the
// cache overflow area for slots >= cache capacity when cache != null).
// Round r of a round-robin CD sweep over n (even) nodes [Alg. 1]; acc: n/2
// doubles of |dW| per pair slot, changes: count of changed couplings.
rec_status rec_launch_cd_round(rec_ctx* ctx, int64_t r, int64_t n, double* acc, int64_t* changes);

// Number of leading positive entries of the descending array g[0, n) (synchronises).
rec_status rec_positive_prefix(rec_ctx* ctx, const double* g, int64_t n, int64_t* np);

// Per-call scratch of the pair-score kernels: the queue of sides the kink
// screen leaves to the exact solver and its counter, the error flags and the
// work counters (may be null).  By default it is carved from the workspace.
struct ScoreScratch {
  uint32_t* queue;
  int64_t* qn;
  int64_t qcap;
  int32_t* err;
  int64_t* work;
  bool fill;   // clear qn with a fill kernel (no memset node) instead of hipMemsetAsync
};
// Score pairs (I, J) into gain_out / w_out with the given scratch, without
// timing events.
rec_status rec_launch_score_with(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                                 double* gain_out, double* w_out, const ScoreScratch& ss);
rec_status rec_launch_score(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                            const uint32_t* slot, double* gain_out, double* w_out,
                            const Cache* cache);
// Score the candidates whose slot word carries the owner bit: pair
// (gi[p], S[v[p]]), gain to the cache slot.
rec_status rec_launch_score_owned(rec_ctx* ctx, int64_t P, const int32_t* gi, const int32_t* v,
                                  const int32_t* S, const uint32_t* slot, const Cache* cache);
// The per-target-row update chains of directed couplings: one wave per
// chain, chains taken in queue order (key/len, n entries; *head zeroed).
rec_status rec_launch_update_chains(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                                    const uint64_t* key, const uint32_t* len, const int32_t* cpair,
                                    int64_t n, int64_t* head, uint8_t* done, double* dw);
// Apply one round of node-disjoint updates: the pairs ready[0..*nready) of
// the rank-ordered list (I, J); at most m of them (see update kernels).
// depth[p] = round for each pair applied.
rec_status rec_launch_update_round(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                                   const int32_t* ready, const int64_t* nready, uint8_t* done,
                                   double* dw, int32_t* depth, int32_t round);
// The pairs of the rank-ordered list (I, J)[0, m) not yet done (done[p] == 0)
// as one dataflow launch over the grid: pair p runs once its predecessors
// pred[2p], pred[2p+1] (or -1) are done.  depth[p] = 1 + the larger depth of
// its predecessors; *rounds receives the largest depth of the pairs it ran.
// *ticket, *rounds and *abort_flag zeroed by the caller.  A wait longer than
// spin_limit polls sets error bit 1024 and ends the launch.
rec_status rec_launch_update_flow(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J, const int32_t* pred,
                                  uint8_t* done, double* dw, int32_t* depth, int64_t* ticket, int64_t* rounds,
                                  int64_t* abort_flag, int64_t spin_limit);

// sort.hip
// Stable LSD radix sort of (khi, klo, val) by the 8-bit digits listed
// (word 0 = klo, 1 = khi; shift in bits), in the given order.
struct Digit { int word, shift; };
rec_status rec_radix_sort(rec_ctx* ctx, int64_t n, const Digit* digits, int nd, int* cur);
rec_status rec_exclusive_scan(rec_ctx* ctx, const int64_t* in, int64_t* out, int64_t n,
                              int64_t* total_dev);

// screen.hip: candidates of the exhaustive screen into ts_i/ts_j (count *n_out)
// for the best m pairs, with nnz current couplings in the compacted W list
// (wi/wj/wv)
rec_status rec_screen_candidates(rec_ctx* ctx, int64_t m, int64_t nnz, int64_t* n_out);
rec_status rec_screen_resolve(rec_ctx* ctx);   // fold finished screen events into sc_stat
// Ising/kinetic, after rec_screen_candidates: append the current couplings
// (wi/wj/wv, nnz) whose gain bound reaches the screen's threshold; *n_out =
// candidates + appended couplings
rec_status rec_screen_couplings(rec_ctx* ctx, int64_t nnz, int64_t* n_out);

// surrogate.hip
rec_status rec_sur_init(rec_ctx* ctx);     // projection bits, initial weights, Adam state
rec_status rec_sur_pack(rec_ctx* ctx);     // bf16 weight copies for inference
rec_status rec_sur_sketch(rec_ctx* ctx);   // sketches at the current state
rec_status rec_sur_infer(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                         const int32_t* Jmap, const uint32_t* slot, float* out);
rec_status rec_sur_grad(rec_ctx* ctx, int64_t B, const int32_t* I, const int32_t* J, const float* y);
rec_status rec_sur_adam(rec_ctx* ctx, float lr);
rec_status rec_sur_filter(rec_ctx* ctx, int64_t n, const int32_t* gi, const int32_t* v,
                          const int32_t* S, uint32_t* slot, int shadow);
rec_status rec_sur_count(rec_ctx* ctx, int64_t n, const uint32_t* slot);
rec_status rec_sur_collect_train(rec_ctx* ctx, double* loss, int64_t* npos, int64_t* nzero);

// search.hip
rec_status rec_search_best(rec_ctx* ctx, int64_t m, int search, int64_t* n_out,
                           rec_sweep_stats* st);
rec_status rec_search_knn(rec_ctx* ctx, int64_t n, const int32_t* S_dev, int k, int level, int mode,
                          int32_t* nbr, double* gain, int* iters);
rec_status rec_apply_best(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                          double* delta, int64_t* accepted, int64_t* rounds);
