// Shared device helpers of the gfx950 reconstruction library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define REC_WAVE 64

// ------------------------------------------------------------------ RNG --
// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014) and the
// counter generator key(seed, stream, a, b) built from it.
__host__ __device__ __forceinline__ uint64_t rec_mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t rec_ctr(uint64_t seed, uint64_t stream, uint64_t a,
                                                     uint64_t b) {
  return rec_mix64(rec_mix64(rec_mix64(rec_mix64(seed) ^ stream) ^ a) ^ b);
}
// floor(r * bound / 2^64): an integer in [0, bound)
__device__ __forceinline__ uint64_t rec_below(uint64_t r, uint64_t bound) {
  return __umul64hi(r, bound);
}

constexpr uint64_t REC_STREAM_INIT = 5;  // NNDescent initial lists
constexpr uint64_t REC_STREAM_CAP = 6;   // in-neighbour sampling of the undirected graph U
constexpr uint64_t REC_STREAM_PROJ = 7;  // +-1 projections of the sketches
constexpr uint64_t REC_STREAM_INIT_W = 8;  // initial MLP weights
constexpr uint64_t REC_STREAM_AUDIT = 9;   // audit and training-record sampling

// learned proposal: sketch width, parameter count, training batch cap
constexpr int REC_SUR_SDIM = 64;
constexpr int64_t REC_SUR_NPARAM = 192 * 128 + 128 + 128 * 128 + 128 + 128 + 1;
constexpr int64_t REC_SUR_BATCH = 8192;

// ------------------------------------------------------------ pair keys --
// Symmetric models: one key per unordered pair; kinetic: ordered (i <- j).
__host__ __device__ __forceinline__ uint64_t rec_pair_key(int i, int j, bool directed) {
  if (!directed && i > j) { int t = i; i = j; j = t; }
  return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j;
}
constexpr uint64_t REC_EMPTY = ~0ULL;

// Order-preserving map of a double to uint64 (ascending) and its inverse.
__host__ __device__ __forceinline__ uint64_t rec_ord(double g) {
  uint64_t u = __builtin_bit_cast(uint64_t, g);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ULL);
}
__host__ __device__ __forceinline__ double rec_unord(uint64_t o) {
  uint64_t u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFULL) : ~o;
  return __builtin_bit_cast(double, u);
}
// key that sorts gains in descending order under an ascending sort
__host__ __device__ __forceinline__ uint64_t rec_desc_key(double g) { return ~rec_ord(g); }
__host__ __device__ __forceinline__ double rec_desc_gain(uint64_t k) { return rec_unord(~k); }

// ----------------------------------------------------------- open hashing --
__device__ __forceinline__ uint64_t rec_hash_slot(uint64_t key, uint64_t mask) {
  return rec_mix64(key) & mask;
}

// Look up key in a linear-probing table; returns the slot or -1.
__device__ __forceinline__ int64_t rec_hash_find(const uint64_t* keys, uint64_t mask, uint64_t key,
                                                 int max_probe) {
  uint64_t s = rec_hash_slot(key, mask);
  for (int p = 0; p < max_probe; ++p) {
    uint64_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
    if (k == key) return (int64_t)s;
    if (k == REC_EMPTY) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

// Insert key if absent.  Returns the slot; *inserted tells whether this call
// created it.  Returns -1 when max_probe slots were all taken by other keys.
__device__ __forceinline__ int64_t rec_hash_insert(uint64_t* keys, uint64_t mask, uint64_t key,
                                                   int max_probe, bool* inserted) {
  uint64_t s = rec_hash_slot(key, mask);
  *inserted = false;
  for (int p = 0; p < max_probe; ++p) {
    uint64_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
    if (k == key) return (int64_t)s;
    if (k == REC_EMPTY) {
      uint64_t prev = atomicCAS((unsigned long long*)&keys[s], (unsigned long long)REC_EMPTY,
                                (unsigned long long)key);
      if (prev == REC_EMPTY) { *inserted = true; return (int64_t)s; }
      if (prev == key) return (int64_t)s;
    }
    s = (s + 1) & mask;
  }
  return -1;
}

// ------------------------------------------------------- wave reductions --
template <class T>
__device__ __forceinline__ T rec_wave_sum(T v) {
  // butterfly: every lane ends with the same bits (each step adds a commuting pair)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, REC_WAVE);
  return v;
}

__device__ __forceinline__ int rec_lane() { return (int)(threadIdx.x & (REC_WAVE - 1)); }

// Values known to be equal on every lane (wave reductions, broadcasts) moved
// to scalar registers, so the compiler treats dependent control flow and
// addressing as uniform.
__device__ __forceinline__ int rec_uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double rec_uni(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T rec_wave_sum_uni(T v) { return rec_uni(rec_wave_sum(v)); }

// Lane q's value of v as a scalar (q uniform): one v_readlane per dword, no
// LDS round trip as a shuffle takes.
__device__ __forceinline__ int rec_lane_val(int v, int q) { return __builtin_amdgcn_readlane(v, q); }
__device__ __forceinline__ double rec_lane_val(double v, int q) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, q);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), q);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Full-wave sums with DPP row operations (xor 1, xor 2, half-row mirror,
// row mirror: every lane of a 16-lane row then holds the row sum) and four
// readlanes for the rows; the result is uniform (scalar).  All 64 lanes must
// be active.  The order of additions is fixed, so the bits do not depend on
// which lane holds which partial sum.
namespace rec_dpp {
constexpr int QP_XOR1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);   // quad_perm [1,0,3,2]
constexpr int QP_XOR2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);   // quad_perm [2,3,0,1]
constexpr int ROW_HALF_MIRROR = 0x141;
constexpr int ROW_MIRROR = 0x140;
template <int CTRL>
__device__ __forceinline__ int mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float mov(float v) {
  return __builtin_bit_cast(float, mov<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double mov(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  int lo = mov<CTRL>((int)(uint32_t)u);
  int hi = mov<CTRL>((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_read(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
}  // namespace rec_dpp

template <class T>
__device__ __forceinline__ T rec_wave_sum_dpp(T v) {
  using namespace rec_dpp;
  v += mov<QP_XOR1>(v);
  v += mov<QP_XOR2>(v);
  v += mov<ROW_HALF_MIRROR>(v);
  v += mov<ROW_MIRROR>(v);
  T r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
  return (r0 + r1) + (r2 + r3);
}

// Append from any subset of a wave's active lanes: one atomic per wave on the
// shared cursor (ballot + popcount ranks), instead of one per lane.  Returns
// the position of this lane's item, or -1 when pred is false.
__device__ __forceinline__ int64_t rec_append(int64_t* cursor, bool pred) {
  uint64_t mask = __ballot(pred);
  if (!pred) return -1;
  const int lane = rec_lane();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  const uint64_t lt = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  long long base = 0;
  if (lane == leader)
    base = (long long)atomicAdd((unsigned long long*)cursor, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader, REC_WAVE);
  return (int64_t)base + __popcll(mask & lt);
}

// Append from the lanes of a whole block (all threads must call): one atomic
// per block on the shared cursor.  sh: NW + 1 ints of LDS, NW = waves per block.
template <int NW>
__device__ __forceinline__ int64_t rec_block_append(int64_t* cursor, bool pred, long long* sh) {
  const int lane = rec_lane(), wave = (int)(threadIdx.x / REC_WAVE);
  uint64_t mask = __ballot(pred);
  const uint64_t lt = lane ? (~0ULL >> (64 - lane)) : 0ULL;
  if (lane == 0) sh[wave] = (long long)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int w = 0; w < NW; ++w) { long long c = sh[w]; sh[w] = tot; tot += c; }
    sh[NW] = tot ? (long long)atomicAdd((unsigned long long*)cursor, (unsigned long long)tot) : 0;
  }
  __syncthreads();
  int64_t pos = pred ? (int64_t)(sh[NW] + sh[wave] + __popcll(mask & lt)) : -1;
  __syncthreads();
  return pos;
}

// Work counters of the pair-score kernel (REC_WORK_N per copy) are kept in
// REC_WORK_COPIES copies so that concurrent waves do not serialise on one
// address; readers sum the copies.  Order: pairs scored, moment passes, full
// evaluations, log passes, sides decided by the residual screen, j-side
// tanh rows fetched, i-side row loads, reserved.
constexpr int REC_WORK_COPIES = 256;
constexpr int REC_WORK_N = 8;

// Residual copies for the screens: int8 q = round(63.5 r), |r| < 2, so
// |q| <= 127.  The value of q is q / 63.5; one term's error |r - q / 63.5| is
// at most 1/127 plus the float product's rounding (2^-24 of 127, < 2^-22 in
// all).
constexpr float REC_Q8_SCALE = 63.5f;
constexpr float REC_Q8_INV = 1.0f / 63.5f;
__device__ __forceinline__ int8_t rec_q8(float r) {
  const float v = rintf(r * REC_Q8_SCALE);
  return (int8_t)fminf(fmaxf(v, -127.f), 127.f);
}

// numerics shared by the kernels (double)
__device__ __forceinline__ double rec_lcosh_tau(double tau) {   // log cosh(atanh tau)
  return -0.5 * log1p(-tau * tau);
}
__device__ __forceinline__ double rec_atanh(double tau) {
  return 0.5 * log1p(2.0 * tau / (1.0 - tau));
}
