// Candidate search: FindBest [Alg. 3] over NNDescent [Alg. 4] or exact KNN,
// the exhaustive top-m, and the update rounds of GCD [Alg. 2].
//
// Within one FindBest level the node set S is held as a sorted array of
// global ids and every KNN list uses local indices into S (so "index asc"
// ties break the same way on local and global ids).
//
// NNDescent, order-independent form: every iteration builds the undirected
// view U of the current lists G (out-neighbours plus at most k in-neighbours
// per node, the k with the smallest (32-bit counter hash, index)), then for
// every node a at once G'[a] = top-k of G[a] and all second neighbours of a
// in U, ranked by (gain desc, index asc) [Alg. 4, parallel per node as in
// App. B].  Scores go through a per-call cache [App. B, caching]: a pair is
// claimed in an open-addressing table the first time it is met and scored
// once; later meetings read the stored gain.
//
// Kinetic model: FindBest needs a symmetric score, so it runs over unordered
// pairs scored by max(gain(i <- j), gain(j <- i)); the best m directed pairs
// are then taken from both directions of the m unordered pairs it returns.
//
// FindBest level: D+ = the 2m best directed edges of G ranked by (gain desc,
// min id, max id, source), D = their unordered pairs, S' = nodes whose every
// out-edge lies in D, recurse on S'; the base case |S|^2 <= 4m scores all
// pairs of S.  D of every level goes to a pool whose best m are returned.
#include <algorithm>
#include <chrono>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"

namespace {

constexpr int BT = 256;

__device__ __forceinline__ bool better(double g1, int i1, double g2, int i2) {
  // NaN ranks last
  if (g1 != g1) return false;
  if (g2 != g2) return true;
  return g1 > g2 || (g1 == g2 && i1 < i2);
}

// Claim a score slot for pair (i, j) (global ids).  A new claim is queued on
// the to-score list.  Returns the value slot (>= table size: overflow area).
struct ClaimArgs {
  Cache C;
  int32_t* ts_i;
  int32_t* ts_j;
  uint32_t* ts_slot;
  int64_t* ts_n;
  int64_t ts_cap;
  int64_t* ovf_n;
  int32_t* err;
  int directed;
};

// Score-cache keys carry, in bits the pair ids leave free (ids < 2^20), the
// search level + 1 at which each endpoint last took the pair as a candidate:
// bits 56..63 for the smaller id, 24..31 for the larger.  A node that meets a
// pair it already merged at this level skips it: its list only improved
// since, so a pair that did not enter then cannot enter now [Alg. 4], and one
// that did is in the list.  Key comparisons mask the tags.
constexpr uint64_t REC_TAG_MASK = 0xFF000000FF000000ULL;

// Insert key (untagged) if absent; *ins tells whether this call created it.
__device__ __forceinline__ int64_t cache_insert(uint64_t* keys, uint64_t mask, uint64_t key,
                                                bool* ins) {
  uint64_t s = rec_hash_slot(key, mask);
  *ins = false;
  for (int p = 0; p < REC_MAX_PROBE; ++p) {
    uint64_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
    if (k == REC_EMPTY) {
      uint64_t prev = atomicCAS((unsigned long long*)&keys[s], (unsigned long long)REC_EMPTY,
                                (unsigned long long)key);
      if (prev == REC_EMPTY) { *ins = true; return (int64_t)s; }
      k = prev;
    }
    if ((k & ~REC_TAG_MASK) == key) return (int64_t)s;
    s = (s + 1) & mask;
  }
  return -1;
}

// The same, setting this endpoint's level tag; *seen tells whether the tag
// already held `tag` (the endpoint took the pair as a candidate at this level).
__device__ __forceinline__ int64_t cache_insert_tag(uint64_t* keys, uint64_t mask, uint64_t key,
                                                    int shift, uint64_t tag, bool* ins, bool* seen) {
  uint64_t s = rec_hash_slot(key, mask);
  const uint64_t tmask = 0xFFull << shift, tval = tag << shift;
  *ins = false;
  *seen = false;
  for (int p = 0; p < REC_MAX_PROBE; ++p) {
    uint64_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
    if (k == REC_EMPTY) {
      uint64_t prev = atomicCAS((unsigned long long*)&keys[s], (unsigned long long)REC_EMPTY,
                                (unsigned long long)(key | tval));
      if (prev == REC_EMPTY) { *ins = true; return (int64_t)s; }
      k = prev;
    }
    if ((k & ~REC_TAG_MASK) == key) {
      while ((k & tmask) != tval) {
        uint64_t prev = atomicCAS((unsigned long long*)&keys[s], (unsigned long long)k,
                                  (unsigned long long)((k & ~tmask) | tval));
        if (prev == k) return (int64_t)s;
        k = prev;   // the other endpoint changed its tag: retry
      }
      *seen = true;
      return (int64_t)s;
    }
    s = (s + 1) & mask;
  }
  return -1;
}

// May be called from any subset of a wave's lanes; the cursors are advanced
// once per wave.
__device__ uint32_t claim(const ClaimArgs& A, int i, int j) {
  bool ins = false;
  int64_t s = cache_insert(A.C.keys, A.C.mask, rec_pair_key(i, j, A.directed != 0), &ins);
  uint64_t slot = s >= 0 ? (uint64_t)s : 0;
  int64_t o = rec_append(A.ovf_n, s < 0);         // no free slot: overflow area
  if (o >= 0) {
    if (o >= A.C.ovf_cap) atomicOr(A.err, 16);
    slot = (A.C.mask + 1) + (uint64_t)o;
  }
  bool queue = s < 0 || ins;                      // this lane scores the pair
  int64_t p = rec_append(A.ts_n, queue);
  if (!queue) return (uint32_t)slot;
  if (p >= A.ts_cap || (s < 0 && o >= A.C.ovf_cap)) { atomicOr(A.err, 16); return 0xffffffffu; }
  A.ts_i[p] = i;
  A.ts_j[p] = j;
  A.ts_slot[p] = (uint32_t)slot;
  return (uint32_t)slot;
}

// Candidate claims mark the lane that must score the pair with the top bit
// of its slot word (REC_OWNER) instead of queueing it, so no shared cursor is
// touched; the score kernel then runs over the candidate array itself.
constexpr uint32_t REC_OWNER = 0x80000000u;
constexpr uint32_t REC_SLOT_BAD = 0x7fffffffu;

// Candidate claim by node i of pair (i, j) at search level `level`.
// *seen: i already took this pair as a candidate at this level (skip it).
__device__ uint32_t claim_owned(const ClaimArgs& A, int i, int j, int level, bool* seen) {
  bool ins = false;
  const uint64_t key = rec_pair_key(i, j, A.directed != 0);
  const int shift = i < j ? 56 : 24;
  int64_t s = cache_insert_tag(A.C.keys, A.C.mask, key, shift, (uint64_t)((level + 1) & 0xff), &ins,
                               seen);
  int64_t o = rec_append(A.ovf_n, s < 0);         // no free slot: overflow area (rare)
  if (s >= 0) return (uint32_t)s | (ins ? REC_OWNER : 0u);
  if (o >= A.C.ovf_cap) { atomicOr(A.err, 16); return REC_SLOT_BAD; }
  return (uint32_t)((A.C.mask + 1) + (uint64_t)o) | REC_OWNER;
}

__device__ __forceinline__ double slot_gain(const Cache& C, uint32_t slot) {
  slot &= ~REC_OWNER;
  if (slot == REC_SLOT_BAD || slot == 0x7fffffffu) return __builtin_nan("");
  uint64_t cap = C.mask + 1;
  return slot < cap ? C.vals[slot] : C.ovf[slot - cap];
}

// ---------------------------------------------------------------- init --
// Random initial list of node a [Alg. 4, first step]: Floyd's sampling of k
// distinct values from the n-1 other local indices, draws from the counter
// generator keyed by (level, global id of a, draw index).
__global__ __launch_bounds__(REC_WAVE) void k_knn_init(const int32_t* S, int64_t n, int k,
                                                       uint64_t seed, int level, int use_bitmap,
                                                       int32_t* cand_v, uint32_t* cand_slot,
                                                       ClaimArgs A) {
  extern __shared__ uint32_t bm[];
  const int64_t a = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t words = (n + 31) / 32;
  if (use_bitmap)
    for (int64_t w = lane; w < words; w += REC_WAVE) bm[w] = 0;
  __syncthreads();
  int32_t* out = cand_v + a * k;
  if (lane == 0) {
    const uint64_t tag = ((uint64_t)(uint32_t)level << 32) | (uint32_t)S[a];
    int c = 0;
    for (int64_t t = (n - 1) - k; t <= n - 2; ++t) {
      int64_t v = (int64_t)rec_below(rec_ctr(seed, REC_STREAM_INIT, tag, (uint64_t)t), (uint64_t)(t + 1));
      bool has;
      if (use_bitmap) has = (bm[v >> 5] >> (v & 31)) & 1u;
      else {
        has = false;
        for (int q = 0; q < c; ++q) {
          int64_t b = out[q];
          int64_t vb = b < a ? b : b - 1;   // back to the value space [0, n-2]
          if (vb == v) { has = true; break; }
        }
      }
      int64_t pick = has ? t : v;
      if (use_bitmap) bm[pick >> 5] |= 1u << (pick & 31);
      out[c++] = (int32_t)(pick < a ? pick : pick + 1);
    }
  }
  __syncthreads();
  for (int c = lane; c < k; c += REC_WAVE) {
    int b = out[c];
    cand_slot[a * k + c] = claim(A, S[a], S[b]);
  }
}

// ------------------------------------------------------------ in-edges --
// Undirected view U: every node b keeps all its out-neighbours and, of its
// in-neighbours a (edges a -> b), the k with the smallest (hash32, a) keys.
// In-neighbours of the KNN graph by target, without atomics: the n k edges
// (record = target, edge index) are sorted by target (stable, so sources
// ascend within a target), each target's range is read off the sorted
// targets, and each in-edge gets its key (hash << 32 | source).  Device-scope
// atomics on random targets (a count, then a cursor per edge) had run at
// about 1.4e9 a second.
__global__ void k_in_records(const int32_t* Gidx, int64_t ne, uint64_t* tgt, uint32_t* eidx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  tgt[e] = (uint64_t)(uint32_t)Gidx[e];
  eidx[e] = (uint32_t)e;
}

// inoff[b] = first sorted position of target b, for b in [0, n]; position p
// writes the targets in (t[p - 1], t[p]] (p = 0: from 0; p = ne: up to n),
// so every entry is written once
__global__ void k_in_bounds(const uint64_t* tgt, int64_t ne, int64_t n, int64_t* inoff) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > ne) return;
  const int64_t lo = p == 0 ? -1 : (int64_t)tgt[p - 1];
  const int64_t hi = p == ne ? n : (int64_t)tgt[p];
  for (int64_t b = lo + 1; b <= hi; ++b) inoff[b] = p;
}

__global__ void k_in_keys(const int32_t* S, const uint64_t* tgt, const uint32_t* eidx, int64_t ne, int k,
                          uint64_t seed, int level, int iter, uint64_t* in_key) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ne) return;
  const int64_t a = (int64_t)eidx[p] / k;
  const int b = (int)tgt[p];
  uint64_t h = rec_ctr(seed, REC_STREAM_CAP, ((uint64_t)(uint32_t)level << 32) | (uint32_t)iter,
                       ((uint64_t)(uint32_t)S[a] << 32) | (uint32_t)S[b]) >> 32;
  in_key[p] = (h << 32) | (uint64_t)a;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, REC_WAVE);
    v = w < v ? w : v;
  }
  return v;
}

// one wave per node (four nodes per block): capin[b*k + c] = sources of the
// (up to) k smallest keys, in increasing key order.  A node's keys (up to
// IN_REG per lane) are read once into registers and the k rounds of wave
// minima run on them; a node with more in-edges (a hub of the KNN graph)
// is read once into per-lane sorted lists.
constexpr int IN_REG = 4;
constexpr int IN_TOP = 32;   // per-lane list of the hub path (k up to 32)
__global__ __launch_bounds__(256) void k_in_select(int64_t n, int k, const int64_t* inoff,
                                                   const uint64_t* in_key, int32_t* capin,
                                                   int32_t* capcnt) {
  const int64_t b = (int64_t)blockIdx.x * (256 / REC_WAVE) + threadIdx.x / REC_WAVE;
  if (b >= n) return;
  const int lane = rec_lane();
  const int64_t e0 = inoff[b], deg = inoff[b + 1] - e0;
  if (deg <= k) {
    for (int64_t c = lane; c < deg; c += REC_WAVE) capin[b * k + c] = (int32_t)(in_key[e0 + c] & 0xffffffffu);
    if (lane == 0) capcnt[b] = (int32_t)deg;
    return;
  }
  uint64_t prev = 0;
  if (deg <= (int64_t)REC_WAVE * IN_REG) {
    // keys are (hash << 32 | source), sources < 2^31: never all ones
    uint64_t kv[IN_REG];
#pragma unroll
    for (int t = 0; t < IN_REG; ++t) {
      const int64_t c = lane + (int64_t)t * REC_WAVE;
      kv[t] = c < deg ? in_key[e0 + c] : ~0ULL;
    }
    for (int r = 0; r < k; ++r) {
      uint64_t best = ~0ULL;
#pragma unroll
      for (int t = 0; t < IN_REG; ++t)
        if ((r == 0 || kv[t] > prev) && kv[t] < best) best = kv[t];
      best = wave_min_u64(best);
      if (lane == 0) capin[b * k + r] = (int32_t)(best & 0xffffffffu);
      prev = best;
    }
  } else if (k <= IN_TOP) {
    // hubs: one pass over the keys, each lane keeping its own IN_TOP smallest
    // in a sorted register list; the k smallest overall are among the lanes'
    // lists, taken by k rounds of wave minima over the list heads (the lane
    // holding the minimum drops its head)
    uint64_t lst[IN_TOP];
#pragma unroll
    for (int t = 0; t < IN_TOP; ++t) lst[t] = ~0ULL;
    for (int64_t c = lane; c < deg; c += REC_WAVE) {
      const uint64_t key = in_key[e0 + c];
      if (key < lst[IN_TOP - 1]) {
#pragma unroll
        for (int t = IN_TOP - 1; t > 0; --t)
          if (key < lst[t]) lst[t] = lst[t - 1] > key ? lst[t - 1] : key;
        if (key < lst[0]) lst[0] = key;
      }
    }
    for (int r = 0; r < k; ++r) {
      const uint64_t best = wave_min_u64(lst[0]);
      if (lane == 0) capin[b * k + r] = (int32_t)(best & 0xffffffffu);
      if (lst[0] == best) {
#pragma unroll
        for (int t = 0; t < IN_TOP - 1; ++t) lst[t] = lst[t + 1];
        lst[IN_TOP - 1] = ~0ULL;
      }
    }
  } else {
    for (int r = 0; r < k; ++r) {
      uint64_t best = ~0ULL;
      for (int64_t c = lane; c < deg; c += REC_WAVE) {
        uint64_t key = in_key[e0 + c];
        if ((r == 0 || key > prev) && key < best) best = key;
      }
      best = wave_min_u64(best);
      if (lane == 0) capin[b * k + r] = (int32_t)(best & 0xffffffffu);
      prev = best;
    }
  }
  if (lane == 0) capcnt[b] = k;
}

// ---------------------------------------------------------- candidates --
// mode 0: second neighbours in U (NNDescent); mode 1: all of S (exact KNN).
// pass 0 counts the distinct candidates of a, pass 1 writes them at off[a]
// (relative to base) and claims their scores.
struct CandArgs {
  const int32_t* S;
  const int32_t* Gidx;
  const int32_t* capin;    // n x k capped in-neighbours
  const int32_t* capcnt;   // n
  int64_t n;
  int k;
  int mode;
};

__device__ __forceinline__ int u_size(const CandArgs& P, int64_t b) { return P.k + P.capcnt[b]; }
__device__ __forceinline__ int u_get(const CandArgs& P, int64_t b, int c) {
  return c < P.k ? P.Gidx[b * P.k + c] : P.capin[b * P.k + (c - P.k)];
}

template <int pass>
__global__ __launch_bounds__(BT) void k_cand(CandArgs P, int level, int64_t a0, int64_t a1,
                                             int64_t* cnt, const int64_t* off, int64_t base,
                                             int32_t* cand_v, int32_t* cand_gi,
                                             uint32_t* cand_slot, ClaimArgs A) {
  extern __shared__ uint32_t sm[];
  const int64_t a = a0 + blockIdx.x;
  if (a >= a1) return;
  const int tid = threadIdx.x;
  const int lane = tid & (REC_WAVE - 1);
  const int64_t words = (P.n + 31) / 32;
  uint32_t* bm = sm;
  int32_t* ul = reinterpret_cast<int32_t*>(sm + words);   // U(a), at most 2k entries
  __shared__ int32_t s_cnt;
  __shared__ int32_t s_nu;
  for (int64_t w = tid; w < words; w += BT) bm[w] = 0;
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  // exclude a and its current list
  if (tid == 0) atomicOr(&bm[a >> 5], 1u << (a & 31));
  if (P.mode == 0)
    for (int c = tid; c < P.k; c += BT) {
      int b = P.Gidx[a * P.k + c];
      atomicOr(&bm[b >> 5], 1u << (b & 31));
    }
  int nu = 0;
  if (P.mode == 0) {
    nu = u_size(P, a);
    for (int c = tid; c < nu; c += BT) ul[c] = u_get(P, a, c);
  }
  if (tid == 0) s_nu = nu;
  __syncthreads();
  const int64_t obase = pass ? off[a] - base : 0;
  const int ga = P.S[a];
  const uint64_t lt = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  // all threads run the same number of rounds so the wave ballots see every lane
  const int64_t total = P.mode == 0 ? (int64_t)s_nu * (2 * P.k) : P.n;
  const int64_t rounds = (total + BT - 1) / BT;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t q = r * BT + tid;
    int v = -1;
    if (q < total) {
      if (P.mode == 0) {
        const int span = 2 * P.k;
        int bi = (int)(q / span), c = (int)(q % span);
        int b = ul[bi];
        if (c < u_size(P, b)) v = u_get(P, b, c);
      } else {
        v = (int)q;
      }
    }
    bool fresh = false;
    if (v >= 0) {
      uint32_t bit = 1u << (v & 31);
      fresh = !(atomicOr(&bm[v >> 5], bit) & bit);
    }
    uint64_t mask = __ballot(fresh);
    int wbase = 0;
    if (lane == 0 && mask) wbase = atomicAdd(&s_cnt, (int)__popcll(mask));
    wbase = __shfl(wbase, 0, REC_WAVE);
    if (pass && fresh) {
      int64_t pos = obase + wbase + __popcll(mask & lt);
      if (pos - obase >= cnt[a]) atomicOr(A.err, 128);   // count pass disagrees
      else {
        bool seen;
        const uint32_t sw = claim_owned(A, ga, P.S[v], level, &seen);
        cand_v[pos] = seen ? -1 : v;   // -1: merged before at this level
        cand_gi[pos] = ga;
        cand_slot[pos] = sw;
      }
    }
  }
  __syncthreads();
  if (pass == 0 && tid == 0) cnt[a] = s_cnt;
}

// Single pass (NNDescent): one block per node collects the node's distinct
// candidates in LDS (at most lcap = min(4k^2, n-1): |U(b)| <= 2k), reserves
// their space with one atomic on a shared cursor, then writes and claims
// them.  off[a]/cnt[a] locate the node's run; the order of the runs depends
// on scheduling, which no result depends on (lists rank by (gain, index),
// every pair's score is the same bits whichever node claims it).
__global__ __launch_bounds__(BT) void k_cand_once(CandArgs P, int level, int64_t a0, int64_t a1, int lcap,
                                                  int64_t* cnt, int64_t* off, int64_t* cursor,
                                                  int64_t cap, int32_t* cand_v, int32_t* cand_gi,
                                                  uint32_t* cand_slot, ClaimArgs A) {
  extern __shared__ uint32_t sm[];
  const int64_t a = a0 + blockIdx.x;
  if (a >= a1) return;
  const int tid = threadIdx.x;
  const int lane = tid & (REC_WAVE - 1);
  const int64_t words = (P.n + 31) / 32;
  uint32_t* bm = sm;
  int32_t* ul = reinterpret_cast<int32_t*>(sm + words);   // U(a): at most 2k entries
  int32_t* lb = ul + 2 * P.k;                              // the node's candidates
  __shared__ int32_t s_cnt;
  __shared__ int32_t s_nu;
  __shared__ long long s_base;
  for (int64_t w = tid; w < words; w += BT) bm[w] = 0;
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  if (tid == 0) atomicOr(&bm[a >> 5], 1u << (a & 31));
  for (int c = tid; c < P.k; c += BT) {
    int b = P.Gidx[a * P.k + c];
    atomicOr(&bm[b >> 5], 1u << (b & 31));
  }
  const int nu = u_size(P, a);
  for (int c = tid; c < nu; c += BT) ul[c] = u_get(P, a, c);
  if (tid == 0) s_nu = nu;
  __syncthreads();
  const uint64_t lt = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  const int span = 2 * P.k;
  const int64_t total = (int64_t)s_nu * span;
  const int64_t rounds = (total + BT - 1) / BT;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t q = r * BT + tid;
    int v = -1;
    if (q < total) {
      int bi = (int)(q / span), c = (int)(q % span);
      int b = ul[bi];
      if (c < u_size(P, b)) v = u_get(P, b, c);
    }
    bool fresh = false;
    if (v >= 0) {
      uint32_t bit = 1u << (v & 31);
      fresh = !(atomicOr(&bm[v >> 5], bit) & bit);
    }
    uint64_t mask = __ballot(fresh);
    int wbase = 0;
    if (lane == 0 && mask) wbase = atomicAdd(&s_cnt, (int)__popcll(mask));
    wbase = __shfl(wbase, 0, REC_WAVE);
    if (fresh) {
      int pos = wbase + __popcll(mask & lt);
      if (pos < lcap) lb[pos] = v;
      else atomicOr(A.err, 128);
    }
  }
  __syncthreads();
  const int nc = s_cnt < lcap ? s_cnt : lcap;
  if (tid == 0) {
    long long b = (long long)atomicAdd((unsigned long long*)cursor, (unsigned long long)nc);
    if (b + nc > cap) { atomicOr(A.err, 16); b = -1; }
    s_base = b;
    off[a] = b < 0 ? 0 : b;
    cnt[a] = b < 0 ? 0 : nc;
  }
  __syncthreads();
  const long long base = s_base;
  if (base < 0) return;
  const int ga = P.S[a];
  for (int c = tid; c < nc; c += BT) {
    const int v = lb[c];
    const int64_t pos = base + c;
    bool seen;
    const uint32_t sw = claim_owned(A, ga, P.S[v], level, &seen);
    cand_v[pos] = seen ? -1 : v;   // -1: merged before at this level
    cand_gi[pos] = ga;
    cand_slot[pos] = sw;
  }
}

// ---------------------------------------------------------------- merge --
// Lists of k <= 64 entries (NNDescent iterations): lane c holds entry c of the
// sorted list.  Candidates come 64 at a time; those better than the current
// k-th are merged at once: each entry's new rank = the entries of both sets
// that beat it (all distinct: candidates exclude the list and each other), and
// the entries ranked below k are placed through LDS.  No per-candidate shift.
__global__ __launch_bounds__(REC_WAVE) void k_merge_small(int64_t a0, int64_t a1, int k,
                                                          const int32_t* Gidx, const double* Ggain,
                                                          int32_t* G2idx, double* G2gain,
                                                          const int64_t* cnt, const int64_t* off,
                                                          int64_t base, const int32_t* cand_v,
                                                          const uint32_t* cand_slot, Cache C,
                                                          int64_t* delta, int32_t* err) {
  __shared__ double sg[REC_WAVE];
  __shared__ int32_t sv[REC_WAVE];
  __shared__ uint8_t sn[REC_WAVE];
  const int64_t a = a0 + blockIdx.x;
  if (a >= a1) return;
  const int lane = threadIdx.x;
  const bool in_list = lane < k;
  double lg = in_list ? Ggain[a * k + lane] : 0.0;
  int li = in_list ? Gidx[a * k + lane] : -1;
  int lnew = 0;
  const int64_t nc = cnt[a];
  const int64_t o0 = off[a] - base;
  for (int64_t q0 = 0; q0 < nc; q0 += REC_WAVE) {
    const int64_t q = q0 + lane;
    double cg = 0.0;
    int cv = -1;
    if (q < nc) {
      cv = cand_v[o0 + q];
      if (cv >= 0) cg = slot_gain(C, cand_slot[o0 + q]);
    }
    const double wg = rec_dpp::lane_read(lg, k - 1);
    const int wi = rec_dpp::lane_read(li, k - 1);
    // a NaN gain marks a pair the learned proposal left unscored: never listed
    const bool cand = cv >= 0 && cg == cg && better(cg, cv, wg, wi);
    uint64_t sur = __ballot(cand);
    if (!sur) continue;
    // ranks: list entry c is beaten by the c entries before it and by the
    // candidates that beat it; a candidate by the list entries and candidates
    // that beat it
    int rl = lane, rc = 0;
    for (int c = 0; c < k; ++c) {
      const double g = rec_dpp::lane_read(lg, c);
      const int v = rec_dpp::lane_read(li, c);
      rc += (cand && better(g, v, cg, cv)) ? 1 : 0;
    }
    uint64_t bits = sur;
    while (bits) {
      const int src = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      const double g = rec_dpp::lane_read(cg, src);
      const int v = rec_dpp::lane_read(cv, src);
      if (in_list && better(g, v, lg, li)) ++rl;
      if (cand && src != lane && better(g, v, cg, cv)) ++rc;
    }
    if (in_list && rl < k) { sg[rl] = lg; sv[rl] = li; sn[rl] = (uint8_t)lnew; }
    if (cand && rc < k) { sg[rc] = cg; sv[rc] = cv; sn[rc] = 1; }
    __syncthreads();
    if (in_list) { lg = sg[lane]; li = sv[lane]; lnew = sn[lane]; }
    __syncthreads();
  }
  // invariant: a list never holds the same neighbour twice
  int dupl = 0;
  for (int c = 0; c < k; ++c) {
    const int v = rec_dpp::lane_read(li, c);
    dupl |= (in_list && lane != c && v == li) ? 1 : 0;
  }
  dupl = rec_wave_sum(dupl);
  if (dupl && lane == 0) atomicOr(err, 64);
  if (in_list) {
    G2gain[a * k + lane] = lg;
    G2idx[a * k + lane] = li;
  }
  const int nnew = rec_wave_sum(in_list ? lnew : 0);
  if (lane == 0 && nnew) atomicAdd((unsigned long long*)delta, (unsigned long long)nnew);
}

// ---- general merge (any k; also the first fill and exact-KNN lists) ----
// G2[a] = top-k of G[a] (unless start_empty) and the candidates of a; one
// wave per node, list kept sorted in LDS; adds |G2[a] \ G[a]| to *delta.
__global__ __launch_bounds__(REC_WAVE) void k_merge(int64_t a0, int64_t a1, int k, int start_empty,
                                                    const int32_t* Gidx, const double* Ggain,
                                                    int32_t* G2idx, double* G2gain,
                                                    const int64_t* cnt, const int64_t* off,
                                                    int64_t base, const int32_t* cand_v,
                                                    const uint32_t* cand_slot, Cache C,
                                                    int64_t* delta, int fixed_count, int32_t* err) {
  extern __shared__ double lg[];
  const int64_t a = a0 + blockIdx.x;
  if (a >= a1) return;
  const int lane = threadIdx.x;
  int32_t* li = reinterpret_cast<int32_t*>(lg + k);
  uint8_t* ln = reinterpret_cast<uint8_t*>(li + k);
  int count = 0;
  if (!start_empty) {
    for (int c = lane; c < k; c += REC_WAVE) {
      lg[c] = Ggain[a * k + c];
      li[c] = Gidx[a * k + c];
      ln[c] = 0;
    }
    count = k;
  }
  __syncthreads();
  const int64_t nc = fixed_count ? fixed_count : cnt[a];
  const int64_t o0 = (fixed_count ? a * (int64_t)fixed_count : off[a]) - base;
  for (int64_t q0 = 0; q0 < nc; q0 += REC_WAVE) {
    int64_t q = q0 + lane;
    bool valid = q < nc;
    double g = 0.0;
    int v = 0;
    if (valid) {
      v = cand_v[o0 + q];
      valid = v >= 0;   // a pair this node merged before at this level
      if (valid) g = slot_gain(C, cand_slot[o0 + q]);
    }
    double wg = count == k ? lg[k - 1] : 0.0;
    int wi = count == k ? li[k - 1] : 0;
    // a NaN gain marks a pair the learned proposal left unscored: never listed
    bool pass = valid && g == g && (count < k || better(g, v, wg, wi));
    uint64_t bal = __ballot(pass);
    while (bal) {
      int src = __ffsll((unsigned long long)bal) - 1;
      bal &= bal - 1;
      double cg = __shfl(g, src, REC_WAVE);
      int cv = __shfl(v, src, REC_WAVE);
      // still better than the current worst?
      if (count == k && !better(cg, cv, lg[k - 1], li[k - 1])) continue;
      // insertion point = number of entries better than (cg, cv)
      int pos = 0;
      for (int c = lane; c < count; c += REC_WAVE) pos += better(lg[c], li[c], cg, cv) ? 1 : 0;
      pos = rec_wave_sum(pos);
      int last = count < k ? count : k - 1;   // highest index written by the shift
      // shift [pos, last) right by one, from the back in wave-sized chunks
      for (int c0 = ((last - 1) / REC_WAVE) * REC_WAVE; c0 >= pos - (pos % REC_WAVE) && last > pos;
           c0 -= REC_WAVE) {
        int c = c0 + lane;
        double tg = 0.0;
        int ti = 0;
        uint8_t tn = 0;
        bool mv = c >= pos && c < last;
        if (mv) { tg = lg[c]; ti = li[c]; tn = ln[c]; }
        __syncthreads();
        if (mv) { lg[c + 1] = tg; li[c + 1] = ti; ln[c + 1] = tn; }
        __syncthreads();
        if (c0 == 0) break;
      }
      if (lane == 0) { lg[pos] = cg; li[pos] = cv; ln[pos] = 1; }
      __syncthreads();
      if (count < k) ++count;
    }
  }
  // invariant: a list never holds the same neighbour twice
  int dupl = 0;
  for (int c = lane; c < count; c += REC_WAVE)
    for (int d = 0; d < c; ++d) dupl |= li[d] == li[c];
  dupl = rec_wave_sum(dupl);
  if (dupl && lane == 0) atomicOr(err, 64);
  int nnew = 0;
  for (int c = lane; c < count; c += REC_WAVE) {
    G2gain[a * k + c] = lg[c];
    G2idx[a * k + c] = li[c];
    nnew += ln[c];
  }
  for (int c = count + lane; c < k; c += REC_WAVE) {   // only when n-1 < k (not used)
    G2gain[a * k + c] = __builtin_nan("");
    G2idx[a * k + c] = -1;
  }
  nnew = rec_wave_sum(nnew);
  if (lane == 0 && !start_empty) atomicAdd((unsigned long long*)delta, (unsigned long long)nnew);
}

// ------------------------------------------------------------ level ops --
// Directed edges a -> G[a][c] as sort records (gain desc, min, max, source).
// klo = (min << (nb+1)) | (max << 1) | (source is max), nb = bits of an id.
__global__ void k_edge_records(const int32_t* S, const int32_t* Gidx, const double* Ggain,
                               int64_t n, int k, int nb, uint64_t* khi, uint64_t* klo,
                               uint32_t* val) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  int64_t a = e / k;
  uint32_t ga = (uint32_t)S[a], gb = (uint32_t)S[Gidx[e]];
  uint32_t lo = ga < gb ? ga : gb, hi = ga < gb ? gb : ga;
  khi[e] = rec_desc_key(Ggain[e]);
  klo[e] = ((uint64_t)lo << (nb + 1)) | ((uint64_t)hi << 1) | (uint64_t)(ga == hi ? 1 : 0);
  val[e] = (uint32_t)e;
}

// D+ = first nsel sorted edges: mark their pairs in D, add new ones to the pool.
__global__ void k_mark_d(const uint64_t* khi, const uint64_t* klo, int64_t nsel, int nb,
                         uint64_t* dkeys, uint64_t dmask, uint64_t* pkeys, uint64_t pmask,
                         uint64_t* pool_hi, uint64_t* pool_lo, int64_t* pool_n, int64_t pool_cap,
                         int32_t* err) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nsel) return;
  uint64_t lo = klo[e];
  uint32_t mn = (uint32_t)(lo >> (nb + 1));
  uint32_t mx = (uint32_t)((lo >> 1) & ((1ULL << nb) - 1));
  uint64_t key = ((uint64_t)mn << 32) | mx;
  bool ins;
  bool ok = rec_hash_insert(dkeys, dmask, key, 4096, &ins) >= 0;
  // unscored pairs (NaN gain) stay out of the pool
  const double g = rec_desc_gain(khi[e]);
  bool pool = g == g;
  if (pool) ok = ok && rec_hash_insert(pkeys, pmask, key, 4096, &ins) >= 0;
  if (!ok) atomicOr(err, 32);
  int64_t p = rec_append(pool_n, pool && ok && ins);
  if (p < 0) return;
  if (p >= pool_cap) { atomicOr(err, 32); return; }
  pool_hi[p] = khi[e];
  pool_lo[p] = key;
}

__global__ void k_saturated(const int32_t* S, const int32_t* Gidx, int64_t n, int k,
                            const uint64_t* dkeys, uint64_t dmask, int64_t* flags) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int all = 1;
  for (int c = 0; c < k && all; ++c) {
    uint64_t key = rec_pair_key(S[a], S[Gidx[a * k + c]], false);
    if (rec_hash_find(dkeys, dmask, key, 4096) < 0) all = 0;
  }
  flags[a] = all;
}

__global__ void k_compact_s(const int32_t* S, const int64_t* flags, const int64_t* pos, int64_t n,
                            int32_t* S2) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a < n && flags[a]) S2[pos[a]] = S[a];
}

// all pairs a < b of S (base case): claim their scores
__global__ __launch_bounds__(BT) void k_allpairs_claim(const int32_t* S, int64_t n, uint32_t* slots,
                                                       ClaimArgs A) {
  const int64_t a = blockIdx.x;
  const int64_t rowbase = a * n - a * (a + 1) / 2;   // pairs of rows < a
  for (int64_t b = a + 1 + threadIdx.x; b < n; b += BT)
    slots[rowbase + (b - a - 1)] = claim(A, S[a], S[b]);
}

__global__ __launch_bounds__(BT) void k_allpairs_pool(const int32_t* S, int64_t n,
                                                      const uint32_t* slots, Cache C,
                                                      uint64_t* pkeys, uint64_t pmask,
                                                      uint64_t* pool_hi, uint64_t* pool_lo,
                                                      int64_t* pool_n, int64_t pool_cap,
                                                      int32_t* err) {
  const int64_t a = blockIdx.x;
  const int64_t rowbase = a * n - a * (a + 1) / 2;
  for (int64_t b = a + 1 + threadIdx.x; b < n; b += BT) {
    double g = slot_gain(C, slots[rowbase + (b - a - 1)]);
    uint64_t key = rec_pair_key(S[a], S[b], false);
    bool ins = false;
    bool ok = true;
    // unscored pairs (NaN gain, left by the learned proposal) stay out of the pool
    if (g == g) ok = rec_hash_insert(pkeys, pmask, key, 4096, &ins) >= 0;
    if (!ok) atomicOr(err, 32);
    int64_t p = rec_append(pool_n, g == g && ok && ins);
    if (p < 0) continue;
    if (p >= pool_cap) { atomicOr(err, 32); continue; }
    pool_hi[p] = rec_desc_key(g);
    pool_lo[p] = key;
  }
}

__global__ void k_pool_to_sort(const uint64_t* ph, const uint64_t* pl, int64_t n, uint64_t* khi,
                               uint64_t* klo, uint32_t* val) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  khi[e] = ph[e];
  klo[e] = pl[e];
  val[e] = 0;
}

__global__ void k_take_best(const uint64_t* khi, const uint64_t* klo, int64_t n, int32_t* oi,
                            int32_t* oj, double* og) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  oi[e] = (int32_t)(klo[e] >> 32);
  oj[e] = (int32_t)(klo[e] & 0xffffffffu);
  og[e] = rec_desc_gain(khi[e]);
}

__global__ void k_iota(int32_t* S, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) S[e] = (int32_t)e;
}

__global__ void k_lists_out(const int32_t* S, const int32_t* Gidx, const double* Ggain,
                            int64_t nk, int32_t* nbr, double* gain) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  int b = Gidx[e];
  nbr[e] = b >= 0 ? S[b] : -1;
  gain[e] = Ggain[e];
}

// ---- exhaustive ----
// pairs of rows [r0, r1): symmetric i < j, kinetic all j != i; enumerated
// row by row into (I, J)
__global__ __launch_bounds__(BT) void k_rowpairs(int64_t r0, int64_t N, int directed,
                                                 const int64_t* roff, int32_t* I, int32_t* J) {
  const int64_t i = r0 + blockIdx.x;
  const int64_t o = roff[blockIdx.x];
  if (directed) {
    for (int64_t j = threadIdx.x; j < N - 1; j += BT) {
      I[o + j] = (int32_t)i;
      J[o + j] = (int32_t)(j < i ? j : j + 1);
    }
  } else {
    for (int64_t j = i + 1 + threadIdx.x; j < N; j += BT) {
      I[o + j - i - 1] = (int32_t)i;
      J[o + j - i - 1] = (int32_t)j;
    }
  }
}

// append scored pairs with gain >= thr after the kept records
__global__ void k_ex_append(const int32_t* I, const int32_t* J, const double* g, int64_t np,
                            double thr, int directed, uint64_t* khi, uint64_t* klo, uint32_t* val,
                            int64_t* n, int64_t cap) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ge = e < np ? g[e] : -__builtin_inf();
  int64_t p = rec_append(n, e < np && ge >= thr);
  if (p < 0 || p >= cap) return;
  khi[p] = rec_desc_key(ge);
  klo[p] = rec_pair_key(I[e], J[e], directed != 0);
  val[p] = 0;
}

// pairs (I, J) as sort records keyed by i (then the original order)
__global__ void k_pack_i(const int32_t* I, const int32_t* J, int64_t n, uint64_t* klo, uint64_t* khi,
                         uint32_t* val) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  klo[e] = ((uint64_t)(uint32_t)I[e] << 32) | (uint32_t)J[e];
  khi[e] = 0;
  val[e] = 0;
}

__global__ void k_unpack_ij(const uint64_t* klo, int64_t n, int32_t* I, int32_t* J) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  I[e] = (int32_t)(klo[e] >> 32);
  J[e] = (int32_t)(klo[e] & 0xffffffffu);
}

// kinetic FindBest result: both directions of each unordered pair
__global__ void k_expand_dir(const int32_t* bi, const int32_t* bj, int64_t n, int32_t* I,
                             int32_t* J) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  I[2 * e] = bi[e];
  J[2 * e] = bj[e];
  I[2 * e + 1] = bj[e];
  J[2 * e + 1] = bi[e];
}

// ---- update rounds ----
// W slot of every pair to apply, inserted (value 0) when absent; a zero entry
// is the same as no entry for every reader of the table.
__global__ void k_reserve(WTable W, const int32_t* I, const int32_t* J, int64_t m, int directed,
                          int64_t* slot, int32_t* err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  bool ins;
  const uint64_t key = rec_pair_key(I[p], J[p], directed);
  int64_t s = rec_hash_insert(W.keys, W.mask, key, REC_MAX_PROBE, &ins);
  if (s < 0) atomicOr(err, 2);
  else {
    rec_wbloom_set(W, key);
    if (ins) W.vals[s] = 0.0;
  }
  slot[p] = s;
}

// Row entries of the pairs to apply: key row << 32 | rank, one per row a
// pair touches (directed pairs: row i only).
__global__ void k_row_entries(const int32_t* I, const int32_t* J, int64_t m, int directed,
                              uint64_t* klo, uint64_t* khi, uint32_t* val) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = directed ? m : 2 * m;
  if (e >= ne) return;
  const int64_t p = directed ? e : e >> 1;
  const int32_t row = (directed || !(e & 1)) ? I[p] : J[p];
  klo[e] = ((uint64_t)(uint32_t)row << 32) | (uint32_t)p;
  khi[e] = 0;
  val[e] = 0;
}

// With the entries sorted by (row, rank): pred[2p + side] = the previous pair
// on the row of that side of pair p, or -1 (side 0: row I[p], 1: row J[p]).
__global__ void k_pred(const uint64_t* klo, int64_t ne, const int32_t* I, int32_t* pred) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const uint64_t k = klo[e];
  const uint32_t row = (uint32_t)(k >> 32);
  const int32_t p = (int32_t)(uint32_t)k;
  const int32_t prev = (e > 0 && (uint32_t)(klo[e - 1] >> 32) == row) ? (int32_t)(uint32_t)klo[e - 1] : -1;
  pred[2 * (int64_t)p + ((uint32_t)I[p] == row ? 0 : 1)] = prev;
}

// Directed pairs, entries sorted by (row, rank): cpair[e] = pair of entry e;
// the entry that starts a row's run gets key (0xFE - min(len - 1, 0xFE)) << 32 | e
// and len[e] = the run's length (a one-byte key that sorts longer chains
// first), every other entry key 0xFF << 32 | e; *maxlen = the longest run,
// which is the number of node-disjoint rounds the same updates would take.
__global__ void k_chain_keys(const uint64_t* ek, int64_t ne, int32_t* cpair, uint64_t* key,
                             uint64_t* khi, uint32_t* len, unsigned long long* maxlen) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const uint64_t k = ek[e];
  const uint32_t row = (uint32_t)(k >> 32);
  cpair[e] = (int32_t)(uint32_t)k;
  const bool start = e == 0 || (uint32_t)(ek[e - 1] >> 32) != row;
  int64_t f = e;
  if (start)
    while (f < ne && (uint32_t)(ek[f] >> 32) == row) ++f;
  const uint64_t n = (uint64_t)(f - e);
  const uint64_t hi = start ? 0xFEull - (n - 1 < 0xFEull ? n - 1 : 0xFEull) : 0xFFull;
  key[e] = (hi << 32) | (uint64_t)e;
  khi[e] = 0;
  len[e] = (uint32_t)n;
  if (start) atomicMax(maxlen, (unsigned long long)n);
}

__global__ void k_iota_i32(int32_t* a, int64_t n, int64_t* count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] = (int32_t)e;
  if (e == 0) *count = n;
}

// Before a round: log the pending count, clear the round's two counters.
__global__ void k_round_begin(const int64_t* npend, int64_t* log, int64_t* nready, int64_t* npend_next) {
  *log = *npend;
  *nready = 0;
  *npend_next = 0;
}

// Split the pending pairs: a pair whose predecessors on its rows are done is
// the earliest pending pair of those rows and joins the round (ready); the
// others stay pending.  A grid-stride loop over the device-side count.
__global__ __launch_bounds__(256) void k_split_ready(const int32_t* pend, const int64_t* npend,
                                                     const int32_t* pred, const uint8_t* done,
                                                     int32_t* ready, int64_t* nready,
                                                     int32_t* pend_next, int64_t* npend_next) {
  const int64_t n = *npend;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + threadIdx.x;
    const bool have = q < n;
    int32_t p = 0;
    bool go = false;
    if (have) {
      p = pend[q];
      const int32_t a = pred[2 * (int64_t)p], b = pred[2 * (int64_t)p + 1];
      go = (a < 0 || done[a]) && (b < 0 || done[b]);
    }
    const int64_t r = rec_append(nready, have && go);
    if (r >= 0) ready[r] = p;
    const int64_t k = rec_append(npend_next, have && !go);
    if (k >= 0) pend_next[k] = p;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

__global__ void k_count_pos(const double* dw, int64_t m, int64_t* cnt) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = (p < m && dw[p] > 0.0) ? 1 : 0;
  c = rec_wave_sum(c);
  if (rec_lane() == 0 && c) atomicAdd((unsigned long long*)cnt, (unsigned long long)c);
}

// Length of the leading run of positive values of g[0, n) (g sorted in
// descending order): the one p with g[p] > 0 and not g[p + 1] > 0 writes p + 1.
__global__ void k_positive_prefix(const double* g, int64_t n, int64_t* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n && g[p] > 0.0 && (p + 1 == n || !(g[p + 1] > 0.0))) *out = p + 1;
}

inline int64_t gridn(int64_t n, int b = 256) { return (n + b - 1) / b; }


// Dynamic LDS a block of the candidate and merge kernels may take: the
// device's per-block maximum (160 KB on gfx950) less room for their static
// variables.
size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 64 * 1024;
  return (size_t)v - 1024;
}

int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) < v) ++b;
  return b < 1 ? 1 : b;
}

inline double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Search {
  rec_ctx* ctx;
  ClaimArgs A;
  int64_t* d_ts_n;
  int64_t* d_ovf_n;
  int64_t* d_delta;
  int64_t* d_pool_n;
  int64_t* d_tmp;
  int64_t* d_cur;
  int64_t nnd_iters = 0;
  int levels = 0;
  int64_t screened = 0;

  explicit Search(rec_ctx* c) : ctx(c) {
    d_ts_n = c->counter + 2;
    d_ovf_n = c->counter + 3;
    d_delta = c->counter + 5;
    d_pool_n = c->counter + 7;
    d_tmp = c->counter + 8;
    d_cur = c->counter + 14;
    A.C = c->C;
    A.ts_i = c->ts_i;
    A.ts_j = c->ts_j;
    A.ts_slot = c->ts_slot;
    A.ts_n = d_ts_n;
    A.ts_cap = c->cand_cap;
    A.ovf_n = d_ovf_n;
    A.err = c->err_flag;
    A.directed = c->cfg.model == REC_KINETIC;
  }

  rec_status get(int64_t* dev, int64_t* host) {
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(host, dev, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      ctx->err = "readback failed";
      return REC_E_HIP;
    }
    return REC_OK;
  }

  rec_status check_err() {
    int32_t e = 0;
    if (hipMemcpyAsync(&e, ctx->err_flag, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      ctx->err = "readback failed";
      return REC_E_HIP;
    }
    if (e & (16 | 32)) {
      ctx->err = "search buffers exhausted (increase workspace)";
      return REC_E_NOMEM;
    }
    if (e & 2) { ctx->err = "W table full (increase max_nnz)"; return REC_E_NOMEM; }
  if (e & 1024) { ctx->err = "update rounds did not drain"; return REC_E_NUMERIC; }
    if (e & 64) { ctx->err = "internal: duplicate neighbour in a merged list"; return REC_E_NUMERIC; }
    if (e & 256) { ctx->err = "screen candidates exceed the candidate buffer"; return REC_E_NOMEM; }
    if (e & 512) { ctx->err = "internal: exact-scoring queue overflow"; return REC_E_NUMERIC; }
    if (e & 128) { ctx->err = "internal: candidate passes disagree"; return REC_E_NUMERIC; }
    if (e) { ctx->err = "device error flag " + std::to_string(e); return REC_E_NUMERIC; }
    return REC_OK;
  }

  void clear_cache() {
    hipMemsetAsync(ctx->C.keys, 0xff, (ctx->C.mask + 1) * sizeof(uint64_t), ctx->stream);
  }

  // Score every pair queued on the to-score list since the last call.
  rec_status flush_scores() {
    int64_t nts = 0;
    rec_status st = get(d_ts_n, &nts);
    if (st != REC_OK) return st;
    if (nts > ctx->cand_cap) { ctx->err = "to-score list overflow"; return REC_E_NOMEM; }
    st = rec_launch_score(ctx, nts, ctx->ts_i, ctx->ts_j, ctx->ts_slot, ctx->C.vals, nullptr,
                          &ctx->C);
    hipMemsetAsync(d_ts_n, 0, sizeof(int64_t), ctx->stream);
    return st;
  }

  // KNN lists of S (n nodes) at a level into Gidx/Ggain (k per node).
  rec_status knn(const int32_t* S, int64_t n, int k, int level, int mode, int* iters) {
    hipStream_t s = ctx->stream;
    const uint64_t seed = ctx->cfg.seed;
    if ((int64_t)k * n > ctx->list_cap) { ctx->err = "KNN lists exceed capacity"; return REC_E_NOMEM; }
    const int64_t words = (n + 31) / 32;
    rec_status st;
    *iters = 0;
    size_t merge_lds = (size_t)k * (8 + 4 + 1) + 16;
    if (merge_lds > lds_limit()) { ctx->err = "k too large for the merge kernel"; return REC_E_INVAL; }
    if (mode == 0) {
      // random initial lists [Alg. 4]
      if (n * (int64_t)k > ctx->cand_cap) { ctx->err = "candidate buffer too small for init"; return REC_E_NOMEM; }
      int use_bm = words * 4 <= 48 * 1024 ? 1 : 0;
      hipLaunchKernelGGL(k_knn_init, dim3(n), dim3(REC_WAVE), use_bm ? words * 4 : 0, s, S, n, k,
                         seed, level, use_bm, ctx->cand_v, ctx->cand_slot, A);
      if ((st = flush_scores()) != REC_OK) return st;
      hipLaunchKernelGGL(k_merge, dim3(n), dim3(REC_WAVE), merge_lds, s, (int64_t)0, n, k, 1,
                         ctx->Gidx, ctx->Ggain, ctx->Gidx, ctx->Ggain, ctx->cnt, ctx->off,
                         (int64_t)0, ctx->cand_v, ctx->cand_slot, ctx->C, d_delta, k, ctx->err_flag);
      if ((st = check_err()) != REC_OK) return st;
    }
    int max_iter = ctx->cfg.nnd_max_iter;
    if (max_iter <= 0) {
      int lg = 0;
      for (double c = 1; c < (double)n; c *= 2.0 * k) ++lg;
      max_iter = 2 * lg + 10;
    }
    const int iters_to_run = mode == 0 ? max_iter : 1;
    CandArgs P{S, ctx->Gidx, ctx->in_src, ctx->capcnt, n, k, mode};
    size_t cand_lds = words * 4 + (mode == 0 ? (size_t)2 * k * 4 : 0);
    if (cand_lds > lds_limit()) { ctx->err = "node set too large for the candidate kernel"; return REC_E_INVAL; }
    for (int it = 0; it < iters_to_run; ++it) {
      P.Gidx = ctx->Gidx;   // the lists ping-pong between two buffers
      if (mode == 0) {
        // undirected view U: the k in-neighbours of each node with the smallest keys
        int64_t ne = n * k;
        hipLaunchKernelGGL(k_in_records, dim3(gridn(std::max<int64_t>(ne, 1))), dim3(256), 0, s, ctx->Gidx, ne,
                           ctx->sb.klo[0], ctx->sb.val[0]);
        Digit dg[4];
        int nd = 0;
        for (int bit = 0; bit < bits_for(n); bit += 8) dg[nd++] = {0, bit};
        int sc = 0;
        if ((st = rec_radix_sort(ctx, ne, dg, nd, &sc)) != REC_OK) return st;
        hipLaunchKernelGGL(k_in_bounds, dim3(gridn(ne + 1)), dim3(256), 0, s, ctx->sb.klo[sc], ne, n, ctx->inoff);
        uint64_t* in_key = ctx->sb.klo[1 - sc];
        hipLaunchKernelGGL(k_in_keys, dim3(gridn(std::max<int64_t>(ne, 1))), dim3(256), 0, s, S, ctx->sb.klo[sc],
                           ctx->sb.val[sc], ne, k, seed, level, it, in_key);
        hipLaunchKernelGGL(k_in_select, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, k, ctx->inoff,
                           in_key, ctx->in_src, ctx->capcnt);
      }
      // NNDescent with the node's candidates fitting LDS: one pass per chunk
      const int64_t lcap = std::min<int64_t>(4 * (int64_t)k * k, n - 1);
      const size_t once_lds = (size_t)words * 4 + (size_t)(2 * k + lcap) * 4;
      if (mode == 0 && once_lds <= lds_limit()) {
        hipMemsetAsync(d_delta, 0, sizeof(int64_t), s);
        const int64_t per = std::max<int64_t>(1, ctx->cand_cap / lcap);
        for (int64_t a0 = 0; a0 < n; a0 += per) {
          const int64_t a1 = std::min(n, a0 + per);
          hipMemsetAsync(d_cur, 0, sizeof(int64_t), s);
          // the overflow area holds the scores of the chunk's candidates that
          // found no cache slot; the chunk's merge is their last reader
          hipMemsetAsync(d_ovf_n, 0, sizeof(int64_t), s);
          hipLaunchKernelGGL(k_cand_once, dim3(a1 - a0), dim3(BT), once_lds, s, P, level, a0, a1, (int)lcap,
                             ctx->cnt, ctx->off, d_cur, ctx->cand_cap, ctx->cand_v, ctx->cand_gi,
                             ctx->cand_slot, A);
          int64_t nch = 0;
          if ((st = get(d_cur, &nch)) != REC_OK) return st;
          if (nch > ctx->cand_cap) { ctx->err = "candidate buffer too small"; return REC_E_NOMEM; }
          if (ctx->sur_mode != 0 &&
              (st = rec_sur_filter(ctx, nch, ctx->cand_gi, ctx->cand_v, S, ctx->cand_slot,
                                   ctx->sur_mode == 1 ? 1 : 0)) != REC_OK) return st;
          if ((st = rec_launch_score_owned(ctx, nch, ctx->cand_gi, ctx->cand_v, S, ctx->cand_slot,
                                           &ctx->C)) != REC_OK) return st;
          if (ctx->sur_mode != 0 && (st = rec_sur_count(ctx, nch, ctx->cand_slot)) != REC_OK) return st;
          if (k <= REC_WAVE)
            hipLaunchKernelGGL(k_merge_small, dim3(a1 - a0), dim3(REC_WAVE), 0, s, a0, a1, k,
                               ctx->Gidx, ctx->Ggain, ctx->Gidx2, ctx->Ggain2, ctx->cnt, ctx->off,
                               (int64_t)0, ctx->cand_v, ctx->cand_slot, ctx->C, d_delta,
                               ctx->err_flag);
          else
            hipLaunchKernelGGL(k_merge, dim3(a1 - a0), dim3(REC_WAVE), merge_lds, s, a0, a1, k, 0,
                               ctx->Gidx, ctx->Ggain, ctx->Gidx2, ctx->Ggain2, ctx->cnt, ctx->off,
                               (int64_t)0, ctx->cand_v, ctx->cand_slot, ctx->C, d_delta, 0,
                               ctx->err_flag);
        }
        if ((st = check_err()) != REC_OK) return st;
        std::swap(ctx->Gidx, ctx->Gidx2);
        std::swap(ctx->Ggain, ctx->Ggain2);
        *iters = it + 1;
        int64_t delta = 0;
        if ((st = get(d_delta, &delta)) != REC_OK) return st;
        if ((double)delta < ctx->cfg.nnd_eps * (double)k * (double)n) break;
        continue;
      }
      // count distinct candidates per node, then offsets
      hipLaunchKernelGGL(k_cand<0>, dim3(n), dim3(BT), cand_lds, s, P, level, (int64_t)0, n, ctx->cnt,
                         ctx->off, (int64_t)0, ctx->cand_v, ctx->cand_gi, ctx->cand_slot, A);
      hipMemsetAsync(ctx->cnt + n, 0, sizeof(int64_t), s);
      if ((st = rec_exclusive_scan(ctx, ctx->cnt, ctx->off, n + 1, nullptr)) != REC_OK) return st;
      std::vector<int64_t> hoff(n + 1);
      if (hipMemcpyAsync(hoff.data(), ctx->off, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { ctx->err = "readback failed"; return REC_E_HIP; }
      hipMemsetAsync(d_delta, 0, sizeof(int64_t), s);
      // node chunks whose candidates fit the buffer
      int64_t a0 = 0;
      while (a0 < n) {
        int64_t a1 = a0 + 1;
        while (a1 < n && hoff[a1 + 1] - hoff[a0] <= ctx->cand_cap) ++a1;
        if (hoff[a1] - hoff[a0] > ctx->cand_cap) { ctx->err = "candidate buffer too small"; return REC_E_NOMEM; }
        int64_t base = hoff[a0];
        hipMemsetAsync(d_ovf_n, 0, sizeof(int64_t), s);   // as above: one chunk's uncached scores
        hipLaunchKernelGGL(k_cand<1>, dim3(a1 - a0), dim3(BT), cand_lds, s, P, level, a0, a1, ctx->cnt,
                           ctx->off, base, ctx->cand_v, ctx->cand_gi, ctx->cand_slot, A);
        const int64_t nch = hoff[a1] - hoff[a0];
        // learned proposal: only the best-ranked fraction keeps its owner bit
        if (ctx->sur_mode != 0 &&
            (st = rec_sur_filter(ctx, nch, ctx->cand_gi, ctx->cand_v, S, ctx->cand_slot,
                                 ctx->sur_mode == 1 ? 1 : 0)) != REC_OK) return st;
        // score the claimed candidates in place (owner bit set)
        if ((st = rec_launch_score_owned(ctx, nch, ctx->cand_gi, ctx->cand_v, S,
                                         ctx->cand_slot, &ctx->C)) != REC_OK) return st;
        if (ctx->sur_mode != 0 && (st = rec_sur_count(ctx, nch, ctx->cand_slot)) != REC_OK) return st;
        hipLaunchKernelGGL(k_merge, dim3(a1 - a0), dim3(REC_WAVE), merge_lds, s, a0, a1, k,
                           mode == 1 ? 1 : 0, ctx->Gidx, ctx->Ggain, ctx->Gidx2, ctx->Ggain2,
                           ctx->cnt, ctx->off, base, ctx->cand_v, ctx->cand_slot, ctx->C, d_delta, 0,
                           ctx->err_flag);
        a0 = a1;
      }
      if ((st = check_err()) != REC_OK) return st;
      std::swap(ctx->Gidx, ctx->Gidx2);
      std::swap(ctx->Ggain, ctx->Ggain2);
      *iters = it + 1;
      if (mode == 0) {
        int64_t delta = 0;
        if ((st = get(d_delta, &delta)) != REC_OK) return st;
        if ((double)delta < ctx->cfg.nnd_eps * (double)k * (double)n) break;
      }
    }
    return REC_OK;
  }

  rec_status pool_add_allpairs(const int32_t* S, int64_t n) {
    hipStream_t s = ctx->stream;
    int64_t np = n * (n - 1) / 2;
    if (np <= 0) return REC_OK;
    if (np > ctx->cand_cap) { ctx->err = "base case larger than candidate buffer"; return REC_E_NOMEM; }
    hipLaunchKernelGGL(k_allpairs_claim, dim3(n), dim3(BT), 0, s, S, n, ctx->cand_slot, A);
    rec_status st = flush_scores();
    if (st != REC_OK) return st;
    hipLaunchKernelGGL(k_allpairs_pool, dim3(n), dim3(BT), 0, s, S, n, ctx->cand_slot, ctx->C,
                       ctx->pset_keys, ctx->pset_mask, ctx->pool_hi, ctx->pool_lo, d_pool_n,
                       ctx->pool_cap, ctx->err_flag);
    return REC_OK;
  }

  // Kinetic model: FindBest runs over unordered pairs under the score
  // max(gain(i <- j), gain(j <- i)); this switches the score kernel and the
  // cache keys to that view for the lifetime of the object.
  struct SymView {
    Search* S;
    explicit SymView(Search* s) : S(s) {
      if (S->ctx->cfg.model == REC_KINETIC) { S->ctx->sym_search = true; S->A.directed = 0; }
    }
    ~SymView() {
      S->ctx->sym_search = false;
      S->A.directed = S->ctx->cfg.model == REC_KINETIC;
    }
  };

  // Kinetic model: the best m directed pairs among both directions of the nb
  // unordered pairs in best_* (exact when those are the exact top m under
  // the max score: at most m unordered pairs reach the m-th best directed gain).
  rec_status directed_best(int64_t nb, int64_t m, int64_t* n_out) {
    hipStream_t s = ctx->stream;
    const int64_t nd = 2 * nb;
    if (nd > ctx->cand_cap || nd > ctx->sb.cap) { ctx->err = "m exceeds capacity"; return REC_E_NOMEM; }
    int32_t* I = ctx->ts_i;
    int32_t* J = ctx->ts_j;
    double* g = ctx->C.ovf;
    if (nb > 0) {
      hipLaunchKernelGGL(k_expand_dir, dim3(gridn(nb)), dim3(256), 0, s, ctx->best_i, ctx->best_j,
                         nb, I, J);
      rec_status st = rec_launch_score(ctx, nd, I, J, nullptr, g, nullptr, nullptr);
      if (st != REC_OK) return st;
    }
    int64_t* d_n = ctx->counter + 9;
    hipMemsetAsync(d_n, 0, sizeof(int64_t), s);
    if (nd > 0)
      hipLaunchKernelGGL(k_ex_append, dim3(gridn(nd)), dim3(256), 0, s, I, J, g, nd,
                         -__builtin_inf(), 1, ctx->sb.khi[0], ctx->sb.klo[0], ctx->sb.val[0], d_n,
                         ctx->sb.cap);
    int cur = 0;
    rec_status st = sort_records(nd, &cur);
    if (st != REC_OK) return st;
    int64_t keep = std::min(nd, m);
    if (keep > ctx->best_cap) { ctx->err = "m exceeds capacity"; return REC_E_NOMEM; }
    if (keep > 0)
      hipLaunchKernelGGL(k_take_best, dim3(gridn(keep)), dim3(256), 0, s, ctx->sb.khi[cur],
                         ctx->sb.klo[cur], keep, ctx->best_i, ctx->best_j, ctx->best_g);
    *n_out = keep;
    return check_err();
  }

  // FindBest [Alg. 3] (mode 0 NNDescent, 1 exact KNN): best m pairs into best_*.
  rec_status find_best(int64_t m, int mode, int64_t* n_out, int64_t level_n[], int levels_max) {
    if (ctx->cfg.model == REC_KINETIC) {
      int64_t nb = 0;
      rec_status st;
      {
        SymView view(this);
        st = find_best_sym(m, mode, &nb, level_n, levels_max);
      }
      if (st != REC_OK) return st;
      return directed_best(nb, m, n_out);
    }
    return find_best_sym(m, mode, n_out, level_n, levels_max);
  }

  rec_status find_best_sym(int64_t m, int mode, int64_t* n_out, int64_t level_n[], int levels_max) {
    hipStream_t s = ctx->stream;
    const int64_t N = ctx->cfg.N;
    clear_cache();
    hipMemsetAsync(ctx->pset_keys, 0xff, (ctx->pset_mask + 1) * 8, s);
    hipMemsetAsync(ctx->counter + 2, 0, sizeof(int64_t) * 8, s);
    hipLaunchKernelGGL(k_iota, dim3(gridn(N)), dim3(256), 0, s, ctx->S, N);
    int32_t* S = ctx->S;
    int32_t* S2 = ctx->S2;
    int64_t n = N;
    rec_status st;
    levels = 0;
    nnd_iters = 0;
    for (int level = 0;; ++level) {
      if (level < levels_max) level_n[level] = n;
      ++levels;
      if (n * n <= 4 * m || n < 2) {
        if ((st = pool_add_allpairs(S, n)) != REC_OK) return st;
        break;
      }
      int64_t kk = ctx->cfg.knn_k_override > 0 ? ctx->cfg.knn_k_override : (4 * m + n - 1) / n;
      if (kk > n - 1) kk = n - 1;
      int k = (int)kk;
      int it = 0;
      if ((st = knn(S, n, k, level, mode, &it)) != REC_OK) return st;
      nnd_iters += it;
      // D+ : the 2m best directed edges
      int64_t ne = n * k;
      int nb = bits_for(N);
      hipLaunchKernelGGL(k_edge_records, dim3(gridn(ne)), dim3(256), 0, s, S, ctx->Gidx, ctx->Ggain,
                         n, k, nb, ctx->sb.khi[0], ctx->sb.klo[0], ctx->sb.val[0]);
      Digit dg[16];
      int nd = 0;
      for (int b = 0; b < 2 * nb + 1; b += 8) dg[nd++] = {0, b};
      for (int b = ctx->fp32 ? 24 : 0; b < 64; b += 8) dg[nd++] = {1, b};
      int cur = 0;
      if ((st = rec_radix_sort(ctx, ne, dg, nd, &cur)) != REC_OK) return st;
      int64_t nsel = std::min<int64_t>(2 * m, ne);
      hipMemsetAsync(ctx->dset_keys, 0xff, (ctx->dset_mask + 1) * 8, s);
      hipLaunchKernelGGL(k_mark_d, dim3(gridn(nsel)), dim3(256), 0, s, ctx->sb.khi[cur],
                         ctx->sb.klo[cur], nsel, nb, ctx->dset_keys, ctx->dset_mask, ctx->pset_keys,
                         ctx->pset_mask, ctx->pool_hi, ctx->pool_lo, d_pool_n, ctx->pool_cap,
                         ctx->err_flag);
      // S' = saturated nodes
      hipLaunchKernelGGL(k_saturated, dim3(gridn(n)), dim3(256), 0, s, S, ctx->Gidx, n, k,
                         ctx->dset_keys, ctx->dset_mask, ctx->cnt);
      if ((st = rec_exclusive_scan(ctx, ctx->cnt, ctx->off, n, d_tmp)) != REC_OK) return st;
      hipLaunchKernelGGL(k_compact_s, dim3(gridn(n)), dim3(256), 0, s, S, ctx->cnt, ctx->off, n, S2);
      int64_t n2 = 0;
      if ((st = get(d_tmp, &n2)) != REC_OK) return st;
      if ((st = check_err()) != REC_OK) return st;
      if (n2 >= n) break;   // cannot happen when n^2 > 4m (|S'| <= n/2); guard only
      std::swap(S, S2);
      n = n2;
    }
    // best m of the pool
    int64_t np = 0;
    if ((st = get(d_pool_n, &np)) != REC_OK) return st;
    if (np > ctx->pool_cap) { ctx->err = "pool overflow"; return REC_E_NOMEM; }
    return sort_pool_take(np, m, n_out);
  }

  rec_status sort_pool_take(int64_t np, int64_t m, int64_t* n_out) {
    hipStream_t s = ctx->stream;
    if (np > 0)
      hipLaunchKernelGGL(k_pool_to_sort, dim3(gridn(np)), dim3(256), 0, s, ctx->pool_hi,
                         ctx->pool_lo, np, ctx->sb.khi[0], ctx->sb.klo[0], ctx->sb.val[0]);
    int cur = 0;
    rec_status st = sort_records(np, &cur);
    if (st != REC_OK) return st;
    int64_t nb = std::min(np, m);
    if (nb > ctx->best_cap) { ctx->err = "m exceeds capacity"; return REC_E_NOMEM; }
    if (nb > 0)
      hipLaunchKernelGGL(k_take_best, dim3(gridn(nb)), dim3(256), 0, s, ctx->sb.khi[cur],
                         ctx->sb.klo[cur], nb, ctx->best_i, ctx->best_j, ctx->best_g);
    *n_out = nb;
    return check_err();
  }

  // sort records (desc gain key, pair key) in sort buffer 0
  rec_status sort_records(int64_t n, int* cur) {
    Digit dg[16];
    int nd = 0;
    int nb = bits_for(ctx->cfg.N);
    for (int b = 0; b < nb; b += 8) dg[nd++] = {0, b};
    for (int b = 0; b < nb; b += 8) dg[nd++] = {0, 32 + b};
    for (int b = ctx->fp32 ? 24 : 0; b < 64; b += 8) dg[nd++] = {1, b};
    *cur = 0;
    return rec_radix_sort(ctx, n, dg, nd, cur);
  }

  // Exhaustive through the screening contraction: candidates from the MFMA
  // screen plus the current couplings, rescored exactly; the best m with
  // positive gain are kept (see screen.hip for why none is missed).  Kinetic
  // pairs are ordered, as in the exhaustive search.
  rec_status screen(int64_t m, int64_t* n_out) {
    hipStream_t s = ctx->stream;
    int64_t nnz = 0;
    rec_status st = rec_wtable_compact(ctx, &nnz);
    if (st != REC_OK) return st;
    int64_t nc = 0;
    if ((st = rec_screen_candidates(ctx, m, nnz, &nc)) != REC_OK) return st;
    if ((st = check_err()) != REC_OK) return st;
    int32_t* I = ctx->ts_i;
    int32_t* J = ctx->ts_j;
    double* g = ctx->C.ovf;
    int64_t np = nc + nnz;
    if (ctx->cfg.model == REC_GAUSS) {
      // every current coupling is rescored
      if (np > ctx->cand_cap) { ctx->err = "screen candidates exceed the buffers"; return REC_E_NOMEM; }
      if (nnz > 0) {
        hipMemcpyAsync(I + nc, ctx->wi, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(J + nc, ctx->wj, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
      }
    } else if ((st = rec_screen_couplings(ctx, nnz, &np)) != REC_OK) {
      return st;
    }
    if (np > ctx->cand_cap || np > ctx->sb.cap) { ctx->err = "screen candidates exceed the buffers"; return REC_E_NOMEM; }
    ctx->sc_stat[7] += (double)np;
    // group the pairs by i (stable radix sort on the i digits): the score
    // kernel then loads each i row once per run of pairs
    if (np > 1) {
      hipLaunchKernelGGL(k_pack_i, dim3(gridn(np)), dim3(256), 0, s, I, J, np, ctx->sb.klo[0],
                         ctx->sb.khi[0], ctx->sb.val[0]);
      Digit dg[4];
      int nd = 0;
      for (int b = 0; b < bits_for(ctx->cfg.N); b += 8) dg[nd++] = {0, 32 + b};
      int cur = 0;
      if ((st = rec_radix_sort(ctx, np, dg, nd, &cur)) != REC_OK) return st;
      hipLaunchKernelGGL(k_unpack_ij, dim3(gridn(np)), dim3(256), 0, s, ctx->sb.klo[cur], np, I, J);
    }
    if ((st = rec_launch_score(ctx, np, I, J, nullptr, g, nullptr, nullptr)) != REC_OK) return st;
    int64_t* d_n = ctx->counter + 9;
    hipMemsetAsync(d_n, 0, sizeof(int64_t), s);
    // keep positive gains only
    if (np > 0)
      hipLaunchKernelGGL(k_ex_append, dim3(gridn(np)), dim3(256), 0, s, I, J, g, np,
                         __builtin_bit_cast(double, (uint64_t)1), ctx->cfg.model == REC_KINETIC ? 1 : 0,
                         ctx->sb.khi[0], ctx->sb.klo[0],
                         ctx->sb.val[0], d_n, ctx->sb.cap);
    int64_t tot = 0;
    if ((st = get(d_n, &tot)) != REC_OK) return st;
    int cur = 0;
    if ((st = sort_records(tot, &cur)) != REC_OK) return st;
    int64_t keep = std::min(tot, m);
    if (keep > ctx->best_cap) { ctx->err = "m exceeds capacity"; return REC_E_NOMEM; }
    if (keep > 0)
      hipLaunchKernelGGL(k_take_best, dim3(gridn(keep)), dim3(256), 0, s, ctx->sb.khi[cur],
                         ctx->sb.klo[cur], keep, ctx->best_i, ctx->best_j, ctx->best_g);
    screened = nc;
    *n_out = keep;
    return check_err();
  }

  // Exhaustive: every pair scored exactly, best m kept (chunks of rows).
  rec_status exhaustive(int64_t m, int64_t* n_out) {
    hipStream_t s = ctx->stream;
    const int64_t N = ctx->cfg.N;
    const int directed = ctx->cfg.model == REC_KINETIC;
    const int64_t cap = ctx->ex_cap;
    int64_t kept = 0;
    double thr = -__builtin_inf();
    std::vector<int64_t> roff;
    int64_t r0 = 0;
    rec_status st;
    int32_t* I = ctx->ts_i;
    int32_t* J = ctx->ts_j;
    double* g = ctx->C.ovf;
    while (r0 < N) {
      roff.assign(1, 0);
      int64_t r1 = r0;
      while (r1 < N) {
        int64_t np = directed ? N - 1 : N - 1 - r1;
        if (roff.back() + np > cap && r1 > r0) break;
        roff.push_back(roff.back() + np);
        ++r1;
      }
      int64_t np = roff.back();
      if (np > cap) { ctx->err = "exhaustive chunk exceeds buffer"; return REC_E_NOMEM; }
      if (np > 0) {
        hipMemcpyAsync(ctx->scan_tmp, roff.data(), sizeof(int64_t) * roff.size(), hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_rowpairs, dim3(r1 - r0), dim3(BT), 0, s, r0, N, directed, ctx->scan_tmp, I, J);
        if ((st = rec_launch_score(ctx, np, I, J, nullptr, g, nullptr, nullptr)) != REC_OK) return st;
        int64_t* d_n = ctx->counter + 9;
        hipMemcpyAsync(d_n, &kept, sizeof(int64_t), hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_ex_append, dim3(gridn(np)), dim3(256), 0, s, I, J, g, np, thr, directed,
                           ctx->sb.khi[0], ctx->sb.klo[0], ctx->sb.val[0], d_n, ctx->sb.cap);
        int64_t tot = 0;
        if ((st = get(d_n, &tot)) != REC_OK) return st;
        if (tot > ctx->sb.cap) { ctx->err = "exhaustive keep buffer overflow"; return REC_E_NOMEM; }
        int cur = 0;
        if ((st = sort_records(tot, &cur)) != REC_OK) return st;
        kept = std::min(tot, m);
        if (cur != 0) {
          hipMemcpyAsync(ctx->sb.khi[0], ctx->sb.khi[1], kept * 8, hipMemcpyDeviceToDevice, s);
          hipMemcpyAsync(ctx->sb.klo[0], ctx->sb.klo[1], kept * 8, hipMemcpyDeviceToDevice, s);
        }
        if (kept == m) {
          uint64_t kh = 0;
          hipMemcpyAsync(&kh, ctx->sb.khi[0] + (m - 1), 8, hipMemcpyDeviceToHost, s);
          hipStreamSynchronize(s);
          thr = rec_desc_gain(kh);
        }
      }
      r0 = r1;
    }
    if (kept > ctx->best_cap) { ctx->err = "m exceeds capacity"; return REC_E_NOMEM; }
    if (kept > 0)
      hipLaunchKernelGGL(k_take_best, dim3(gridn(kept)), dim3(256), 0, s, ctx->sb.khi[0],
                         ctx->sb.klo[0], kept, ctx->best_i, ctx->best_j, ctx->best_g);
    *n_out = kept;
    return check_err();
  }
};

}  // namespace

rec_status rec_positive_prefix(rec_ctx* ctx, const double* g, int64_t n, int64_t* np) {
  *np = 0;
  if (n <= 0) return REC_OK;
  int64_t* d = ctx->counter + 15;
  if (hipMemsetAsync(d, 0, sizeof(int64_t), ctx->stream) != hipSuccess) return REC_E_HIP;
  hipLaunchKernelGGL(k_positive_prefix, dim3(gridn(n)), dim3(256), 0, ctx->stream, g, n, d);
  if (hipMemcpyAsync(np, d, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
    return REC_E_HIP;
  return hipStreamSynchronize(ctx->stream) == hipSuccess ? REC_OK : REC_E_HIP;
}

// FindBest over NNDescent with the learned proposal.  Active (the network is
// trained and its last recall estimate reaches the bar): each chunk's
// candidates are ranked and only the top fraction rho is scored, plus an
// audit sample of the rest (1 in sur_audit, by pair hash) from which the
// recall of positive gains is estimated.  Otherwise (fallback): the plain
// search, with the network run in shadow to measure the recall it would have
// had.  Either way the exact scores of this call then train the network.
namespace {
rec_status surrogate_find_best(rec_ctx* ctx, Search& S, int64_t m, int64_t* n_out, int64_t* level_n) {
  hipStream_t s = ctx->stream;
  rec_status r = rec_sur_sketch(ctx);
  if (r != REC_OK) return r;
  const bool active = ctx->sur_trained && ctx->sur_recall >= ctx->sur_recall_min;
  ctx->sur_mode = active ? 2 : 1;
  hipMemsetAsync(ctx->sur_cnt, 0, 16 * sizeof(int64_t), s);
  r = S.find_best(m, 0, n_out, level_n, 64);
  ctx->sur_mode = 0;
  if (r != REC_OK) return r;
  int64_t c[8];
  if (hipMemcpyAsync(c, ctx->sur_cnt, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) { ctx->err = "readback failed"; return REC_E_HIP; }
  // c: kept positives, below-threshold positives (scored), kept, below scored, dropped
  const double scale = active ? (double)ctx->sur_audit : 1.0;
  const double miss = scale * (double)c[1];
  const double est = (c[0] + miss) > 0 ? (double)c[0] / ((double)c[0] + miss) : 1.0;
  const double owned = (double)(c[2] + c[3] + c[4]);
  double loss = 0.0;
  int64_t np = 0, nz = 0;
  if ((r = rec_sur_collect_train(ctx, &loss, &np, &nz)) != REC_OK) return r;
  ctx->sur_trained = true;
  ctx->sur_recall = est;
  double* o = ctx->sur_stats;
  o[0] = active ? 2 : 1;
  o[1] = est;
  o[2] = owned > 0 ? (double)(c[2] + c[3]) / owned : 0.0;   // fraction scored exactly
  o[3] = (double)c[0];
  o[4] = miss;
  o[5] = (double)np;
  o[6] = (double)nz;
  o[7] = loss;
  o[8] = ctx->sur_stats[8] + 1;
  o[9] = ctx->sur_rho;
  return REC_OK;
}
}  // namespace

rec_status rec_search_best(rec_ctx* ctx, int64_t m, int search, int64_t* n_out,
                           rec_sweep_stats* st) {
  Search S(ctx);
  // pair scores so far (the work counters are cumulative)
  int64_t w0[REC_WORK_N] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (st && rec_work_read(ctx, w0) != REC_OK) return REC_E_HIP;
  int64_t level_n[64];
  rec_status r;
  if (search == REC_SEARCH_EXHAUSTIVE) {
    r = S.exhaustive(m, n_out);
  } else if (search == REC_SEARCH_SCREEN) {
    r = S.screen(m, n_out);
  } else if (search == REC_SEARCH_SURROGATE) {
    r = surrogate_find_best(ctx, S, m, n_out, level_n);
  } else if (search == REC_SEARCH_GRADIENT) {
    // FindBest over NNDescent with every search score the absolute gradient
    ctx->grad_dist = true;
    r = S.find_best(m, 0, n_out, level_n, 64);
    ctx->grad_dist = false;
  } else {
    r = S.find_best(m, search == REC_SEARCH_EXACT_KNN ? 1 : 0, n_out, level_n, 64);
  }
  if (r != REC_OK) return r;
  ctx->last_levels = 0;
  if (search != REC_SEARCH_EXHAUSTIVE && search != REC_SEARCH_SCREEN) {
    ctx->last_levels = (int32_t)std::min<int64_t>(S.levels, 64);
    for (int l = 0; l < ctx->last_levels; ++l) ctx->last_level_n[l] = level_n[l];
  }
  if (st) {
    int64_t w1[REC_WORK_N];
    if (rec_work_read(ctx, w1) != REC_OK) return REC_E_HIP;
    st->pair_evals = w1[0] - w0[0];
    st->nnd_iters = S.nnd_iters;
    st->levels = S.levels;
  }
  return REC_OK;
}

rec_status rec_search_knn(rec_ctx* ctx, int64_t n, const int32_t* S_dev, int k, int level, int mode,
                          int32_t* nbr, double* gain, int* iters) {
  Search S(ctx);
  S.clear_cache();
  hipMemsetAsync(ctx->counter + 2, 0, sizeof(int64_t) * 8, ctx->stream);
  rec_status r;
  {
    Search::SymView view(&S);   // kinetic: lists under the max of both directions
    r = S.knn(S_dev, n, k, level, mode, iters);
  }
  if (r != REC_OK) return r;
  hipLaunchKernelGGL(k_lists_out, dim3(gridn(n * k)), dim3(256), 0, ctx->stream, S_dev, ctx->Gidx,
                     ctx->Ggain, n * k, nbr, gain);
  return hipGetLastError() == hipSuccess ? REC_OK : REC_E_HIP;
}

// After the updates of m pairs: Σ|Δw| and the number of changed couplings
// (and, when given, a device count read back with them); synchronises.
static rec_status finish_updates(rec_ctx* ctx, int64_t m, double* delta, int64_t* accepted,
                                 const int64_t* extra_dev, int64_t* extra = nullptr) {
  hipStream_t s = ctx->stream;
  ++ctx->w_version;   // the updates changed W
  if (rec_sum_device(ctx, ctx->dw, m, ctx->dresult + 3) != REC_OK) return REC_E_HIP;
  hipMemsetAsync(ctx->counter + 11, 0, sizeof(int64_t), s);
  hipLaunchKernelGGL(k_count_pos, dim3(gridn(m)), dim3(256), 0, s, ctx->dw, m, ctx->counter + 11);
  hipMemcpyAsync(delta, ctx->dresult + 3, sizeof(double), hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(accepted, ctx->counter + 11, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (extra_dev) hipMemcpyAsync(extra, extra_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  int32_t e = 0;
  hipMemcpyAsync(&e, ctx->err_flag, 4, hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) { ctx->err = "sync failed"; return REC_E_HIP; }
  if (e & 2) { ctx->err = "W table full (increase max_nnz)"; return REC_E_NOMEM; }
  if (e & 1024) { ctx->err = "update rounds did not drain"; return REC_E_NUMERIC; }
  return REC_OK;
}

// Directed couplings: with the row entries (one per pair, row = target)
// sorted by (row, rank) in sort buffer cur, every target row's pairs form a
// chain that only that row's fields see, so running each chain in rank
// order is the sequential order [Alg. 2].  The chains are queued longest
// first (one 8-bit digit of the radix sort, stable in position) and one
// launch runs them all; the reported round count is the longest chain,
// the rounds the node-disjoint schedule would take.
static rec_status apply_chains(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J, int cur,
                               double* delta, int64_t* accepted, int64_t* rounds) {
  hipStream_t s = ctx->stream;
  const int64_t ne = m;
  int32_t* cpair = ctx->pred;   // 2m entries; the chains take m
  int64_t* head = ctx->counter + 0;
  int64_t* maxlen = ctx->counter + 1;
  hipMemsetAsync(ctx->counter, 0, 2 * sizeof(int64_t), s);
  const int o = cur ^ 1;
  hipLaunchKernelGGL(k_chain_keys, dim3(gridn(ne)), dim3(256), 0, s, ctx->sb.klo[cur], ne, cpair,
                     ctx->sb.klo[o], ctx->sb.khi[o], ctx->sb.val[o],
                     reinterpret_cast<unsigned long long*>(maxlen));
  Digit dg[1] = {{0, 32}};
  int c = o;
  rec_status st = rec_radix_sort(ctx, ne, dg, 1, &c);
  if (st != REC_OK) return st;
  st = rec_launch_update_chains(ctx, m, I, J, ctx->sb.klo[c], ctx->sb.val[c], cpair, ne, head,
                                ctx->done, ctx->dw);
  if (st != REC_OK) return st;
  return finish_updates(ctx, m, delta, accepted, maxlen, rounds);
}

// Coordinate updates of the m pairs in rank order [Alg. 2], as rounds of
// node-disjoint pairs (a pair runs once every earlier pair sharing a row
// with it has run), which reproduces the sequential order exactly.  Each
// pair's predecessor on each of its rows comes from one sort of its row
// entries; a round takes the pending pairs whose predecessors are done.
rec_status rec_apply_best(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                          double* delta, int64_t* accepted, int64_t* rounds) {
  hipStream_t s = ctx->stream;
  const int directed = ctx->cfg.model == REC_KINETIC;
  *delta = 0.0;
  *accepted = 0;
  *rounds = 0;
  if (m <= 0) return REC_OK;
  if (m > ctx->best_cap) { ctx->err = "too many pairs for the update buffers"; return REC_E_NOMEM; }
  const int64_t ne = directed ? m : 2 * m;
  if (ne > ctx->sb.cap) { ctx->err = "too many pairs for the sort buffers"; return REC_E_NOMEM; }
  hipMemsetAsync(ctx->done, 0, m, s);
  ctx->w_any = true;   // the reserved slots are W entries
  hipLaunchKernelGGL(k_reserve, dim3(gridn(m)), dim3(256), 0, s, ctx->W, I, J, m, directed, ctx->best_slot,
                     ctx->err_flag);
  // predecessors on the rows
  hipLaunchKernelGGL(k_fill_i32, dim3(gridn(2 * m)), dim3(256), 0, s, ctx->pred, 2 * m, -1);
  hipLaunchKernelGGL(k_row_entries, dim3(gridn(ne)), dim3(256), 0, s, I, J, m, directed, ctx->sb.klo[0],
                     ctx->sb.khi[0], ctx->sb.val[0]);
  {
    // the entries are written in rank order and the radix sort is stable,
    // so the row digits alone give (row, rank) order
    Digit dg[4];
    int nd = 0;
    for (int b = 0; b < bits_for(ctx->cfg.N); b += 8) dg[nd++] = {0, 32 + b};
    int cur = 0;
    rec_status st = rec_radix_sort(ctx, ne, dg, nd, &cur);
    if (st != REC_OK) return st;
    if (directed) return apply_chains(ctx, m, I, J, cur, delta, accepted, rounds);
    hipLaunchKernelGGL(k_pred, dim3(gridn(ne)), dim3(256), 0, s, ctx->sb.klo[cur], ne, I, ctx->pred);
  }
  // pending lists (ping-pong) and their counts, the round's ready count
  int64_t* npend[2] = {ctx->counter + 0, ctx->counter + 1};
  int64_t* d_ready = ctx->counter + 10;
  hipLaunchKernelGGL(k_iota_i32, dim3(gridn(m)), dim3(256), 0, s, ctx->pend[0], m, npend[0]);
  const unsigned split_grid = (unsigned)std::min<int64_t>(gridn(m), 1024);
  int cur = 0;
  int64_t pass = 0;      // rounds that ran pairs
  int32_t launched = 0;  // rounds launched (the empty ones after the last come last)
  // Rounds over the whole grid while they ready many pairs each; once a round
  // readies fewer than flow_min, the pairs left run as one dataflow launch
  // without three launches a round (the runs of updates on hub rows take as
  // many rounds as the hub has pairs).
  const int64_t flow_min = 256;
  while (true) {
    const int batch = 8;
    std::vector<int64_t> rem(batch + 1, 0);
    for (int b = 0; b < batch; ++b) {
      hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, s, npend[cur], ctx->scan_tmp + b, d_ready,
                         npend[cur ^ 1]);
      hipLaunchKernelGGL(k_split_ready, dim3(split_grid), dim3(256), 0, s, ctx->pend[cur], npend[cur], ctx->pred,
                         ctx->done, ctx->ready, d_ready, ctx->pend[cur ^ 1], npend[cur ^ 1]);
      rec_status st = rec_launch_update_round(ctx, m, I, J, ctx->ready, d_ready, ctx->done, ctx->dw, ctx->depth,
                                              ++launched);
      if (st != REC_OK) return st;
      cur ^= 1;
    }
    if (hipMemcpyAsync(rem.data(), ctx->scan_tmp, sizeof(int64_t) * batch, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(rem.data() + batch, npend[cur], sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { ctx->err = "readback failed"; return REC_E_HIP; }
    for (int b = 0; b < batch; ++b)
      if (rem[b] > 0) ++pass;
    if (rem[batch] == 0) break;
    // the earliest pending pair is always ready, so m rounds always suffice
    if (pass > m + batch) { ctx->err = "update rounds did not drain"; return REC_E_NUMERIC; }
    if (rem[batch - 1] - rem[batch] < flow_min) {
      // ticket, depth maximum and abort flag: counter slots the rounds no longer use
      int64_t* ticket = ctx->counter + 0;
      int64_t* d_depth = ctx->counter + 1;
      int64_t* abort_flag = ctx->counter + 14;
      hipMemsetAsync(ticket, 0, 2 * sizeof(int64_t), s);
      hipMemsetAsync(abort_flag, 0, sizeof(int64_t), s);
      rec_status st = rec_launch_update_flow(ctx, m, I, J, ctx->pred, ctx->done, ctx->dw, ctx->depth, ticket,
                                             d_depth, abort_flag, ctx->flow_spin_limit);
      if (st != REC_OK) return st;
      int64_t tail = 0;
      if (hipMemcpyAsync(&tail, d_depth, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { ctx->err = "readback failed"; return REC_E_HIP; }
      pass = std::max(pass, tail);
      break;
    }
  }
  *rounds = pass;
  return finish_updates(ctx, m, delta, accepted, nullptr);
}
