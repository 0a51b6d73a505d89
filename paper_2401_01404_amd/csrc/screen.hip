// Exhaustive screening contraction on the matrix cores.
//
// Gaussian model: for every pair at once, a_ij = x_i . r_j + r_i . x_j is one
// entry of S = A B^T with A_i = [x_i | r_i] and B_j = [r_j | x_j] (K = 2M,
// padded to a multiple of 32 with zeros), r the residuals of the Gaussian
// pseudolikelihood [App. A].  The closed-form gain of a pair at w0 = 0 is
// (|a| - lambda)^2 / (2 b) for |a| > lambda, else 0, with
// b = theta_i^2 |x_j|^2 + theta_j^2 |x_i|^2 (the score kernel's formula).
//
// S is formed in BF16 on MFMA with FP32 accumulation, so a carries an error
// bounded by e_ij = c |A_i| |B_j|: each operand rounds to bf16 with relative
// error <= 2^-8, a product of two by <= 2^-7 + 2^-16, and the fp32 sums add
// <= K 2^-24 of sum |A_k B_k| <= |A_i| |B_j| (Cauchy-Schwarz).  From it every
// pair gets bounds g_lo <= gain <= g_up.  Pass 0 histograms g_lo; tau = the
// lower edge of the bin holding the (m + nnz)-th largest g_lo is a lower bound
// on the m-th best exact gain (at most nnz pairs carry w0 != 0, for which the
// w0 = 0 formula does not hold).  Pass 1 keeps the w0 = 0 pairs with
// g_up >= tau and g_up > 0; they and the current nonzero couplings are then
// rescored by the exact score kernel.  The result equals the exhaustive
// search's positive-gain top m: the screen drops no pair that could reach it.
//
// Ising and kinetic models: the same two passes over an int8 contraction of
// the +-1 samples with the int8 residual copies, with gain bounds from the
// curvature of the log-cosh terms (see the second half of this file).
#include <math.h>
#include <string.h>

#include "common.hpp"
#include "ctx.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer descriptor on gfx9-family GPUs (32-bit data, no swizzle)
constexpr int KS_RSRC3 = 0x00020000;

constexpr int SC_T = 128;      // output tile (rows and columns)
constexpr int SC_K = 32;       // k step of one MFMA
constexpr int SC_LD = 40;      // LDS row stride in bf16 (80 bytes: 16-byte aligned, staggered banks)
constexpr int SC_BINS = 4096;  // histogram bins: the top 12 bits of a positive float

// A_i = [x_i | r_i], B_i = [r_i | x_i] in bf16 (zeros past 2M), the row norm
// |A_i| = |B_i| rounded up, theta_i^2 and |x_i|^2 as floats.
template <class R>
__global__ __launch_bounds__(256) void k_screen_prep(Fields F, int Kp, __bf16* __restrict__ A,
                                                     __bf16* __restrict__ B, float* __restrict__ nrm,
                                                     float* __restrict__ th2, float* __restrict__ sqf) {
  __shared__ double sh[4];
  const int64_t i = blockIdx.x;
  const R* H = reinterpret_cast<const R*>(F.H) + i * F.Mp;
  const float* X = F.xf + i * F.Mp;
  const int64_t M = F.M;
  double s2 = 0.0;
  for (int64_t k = threadIdx.x; k < Kp; k += blockDim.x) {
    double va = 0.0, vb = 0.0;
    if (k < M) { va = X[k]; vb = (double)H[k]; }
    else if (k < 2 * M) { va = (double)H[k - M]; vb = X[k - M]; }
    A[i * Kp + k] = (__bf16)(float)va;
    B[i * Kp + k] = (__bf16)(float)vb;
    s2 += va * va;
  }
  s2 = rec_wave_sum(s2);
  if ((threadIdx.x & (REC_WAVE - 1)) == 0) sh[threadIdx.x / REC_WAVE] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / REC_WAVE); ++w) t += sh[w];
    nrm[i] = (float)(sqrt(t) * (1.0 + 1e-6));
    th2[i] = (float)(F.theta[i] * F.theta[i]);
    sqf[i] = (float)F.sq[i];
  }
}

struct ScreenArgs {
  const __bf16* A;
  const __bf16* B;
  int64_t N;
  int Kp;
  const float* nrm;
  const float* th2;
  const float* sqf;
  float lam;       // lambda (float)
  float cerr;      // e_ij = cerr |A_i| |B_j| + elam
  float elam;      // lambda's rounding and the exact kernel's own rounding
  uint32_t* hist;  // SC_BINS counters (pass 0)
  const float* tau;  // pass 1 threshold (device)
  WTable W;
  int32_t* oi;
  int32_t* oj;
  int64_t* cursor;
  int64_t cap;
  int32_t* err;
};

__device__ __forceinline__ void gain_bounds(const ScreenArgs& P, float a, int64_t i, int64_t j,
                                            float* glo, float* gup) {
  const float e = P.cerr * P.nrm[i] * P.nrm[j] + P.elam;
  const float b = P.th2[i] * P.sqf[j] + P.th2[j] * P.sqf[i];
  const float aa = fabsf(a);
  const float dl = aa - e - P.lam, du = aa + e - P.lam;
  // b and the quotient in float: relative slack 1e-5 either way
  *glo = dl > 0.f ? dl * dl / (2.f * b) * (1.f - 1e-5f) : 0.f;
  *gup = du > 0.f ? du * du / (2.f * b) * (1.f + 1e-5f) : 0.f;
}

// One 128 x 128 tile of S per block (4 waves, 64 x 64 each as 4 x 4 MFMA
// 16x16x32 blocks); only tiles on or above the diagonal run.
template <int PASS>
__global__ __launch_bounds__(256) void k_screen(ScreenArgs P) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  __shared__ __attribute__((aligned(16))) __bf16 As[SC_T * SC_LD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[SC_T * SC_LD];
  __shared__ uint32_t hs[PASS == 0 ? SC_BINS : 1];
  const int tid = threadIdx.x, lane = tid & (REC_WAVE - 1), w = tid / REC_WAVE;
  const int64_t r0 = (int64_t)bi * SC_T, c0 = (int64_t)bj * SC_T;
  if (PASS == 0)
    for (int q = tid; q < SC_BINS; q += 256) hs[q] = 0;
  floatx4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // 128 rows x 32 bf16 per matrix and step = 512 chunks of 16 bytes, two per
  // thread; the next step's chunks are loaded into registers while this
  // step's MFMAs run (the global latency is not on every step's path)
  uint4 va[2], vb[2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = tid + 256 * h, row = q >> 2, ch = q & 3;
      const int64_t ga = r0 + row, gb = c0 + row;
      va[h] = make_uint4(0u, 0u, 0u, 0u);
      vb[h] = make_uint4(0u, 0u, 0u, 0u);
      if (ga < P.N) va[h] = *reinterpret_cast<const uint4*>(P.A + ga * P.Kp + k0 + ch * 8);
      if (gb < P.N) vb[h] = *reinterpret_cast<const uint4*>(P.B + gb * P.Kp + k0 + ch * 8);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < P.Kp; k0 += SC_K) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = tid + 256 * h, row = q >> 2, ch = q & 3;
      *reinterpret_cast<uint4*>(As + row * SC_LD + ch * 8) = va[h];
      *reinterpret_cast<uint4*>(Bs + row * SC_LD + ch * 8) = vb[h];
    }
    __syncthreads();
    if (k0 + SC_K < P.Kp) fetch(k0 + SC_K);
    bf16x8 af[4], bf[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      af[m] = *reinterpret_cast<const bf16x8*>(As + (wr + m * 16 + (lane & 15)) * SC_LD + (lane >> 4) * 8);
#pragma unroll
    for (int n = 0; n < 4; ++n)
      bf[n] = *reinterpret_cast<const bf16x8*>(Bs + (wc + n * 16 + (lane & 15)) * SC_LD + (lane >> 4) * 8);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bf[n], acc[m][n], 0, 0, 0);
    __syncthreads();
  }
  // epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16x16 block
  const float tau = PASS == 1 ? *P.tau : 0.f;
  uint64_t kept = 0;   // pass 1: bit (m, n, r) = 16 m + 4 n + r, the element's upper bound reaches tau
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + wr + m * 16 + 4 * (lane >> 4) + r;
        const int64_t j = c0 + wc + n * 16 + (lane & 15);
        const bool ok = i < j && j < P.N;
        float glo = 0.f, gup = 0.f;
        if (ok) gain_bounds(P, acc[m][n][r], i, j, &glo, &gup);
        if (PASS == 0) {
          if (glo > 0.f) atomicAdd(&hs[__builtin_bit_cast(uint32_t, glo) >> 19], 1u);
        } else if (gup > 0.f && gup >= tau) {
          kept |= 1ull << (16 * m + 4 * n + r);
        }
      }
  // pass 1: the few kept elements (about 2e-3 of them) go to the list, one
  // per lane per round, as many rounds as the fullest lane has elements
  if (PASS == 1) {
    while (__ballot(kept != 0ull)) {
      bool keep = kept != 0ull;
      const int b = keep ? __builtin_ctzll(kept) : 0;
      kept &= kept - 1;
      const int64_t i = r0 + wr + (b >> 4) * 16 + 4 * (lane >> 4) + (b & 3);
      const int64_t j = c0 + wc + ((b >> 2) & 3) * 16 + (lane & 15);
      if (keep && P.W.keys != nullptr) {
        // a current (nonzero) coupling is rescored from the W list instead
        int64_t ws = rec_hash_find(P.W.keys, P.W.mask, rec_pair_key((int)i, (int)j, false), REC_MAX_PROBE);
        if (ws >= 0 && P.W.vals[ws] != 0.0) keep = false;
      }
      int64_t pos = rec_append(P.cursor, keep);
      if (pos >= 0) {
        if (pos < P.cap) {
          P.oi[pos] = (int32_t)i;
          P.oj[pos] = (int32_t)j;
        } else {
          atomicOr(P.err, 256);
        }
      }
    }
  }
  if (PASS == 0) {
    __syncthreads();
    for (int q = tid; q < SC_BINS; q += 256)
      if (hs[q]) atomicAdd(&P.hist[q], hs[q]);
  }
}

// tau = lower edge of the bin holding the target-th largest g_lo (0 if fewer)
__global__ void k_screen_tau(const uint32_t* hist, int64_t target, float* tau) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t cum = 0;
  float t = 0.f;
  for (int q = SC_BINS - 1; q >= 1; --q) {
    cum += hist[q];
    if (cum >= target) { t = __builtin_bit_cast(float, (uint32_t)q << 19); break; }
  }
  *tau = t;
}


// ---------------------------------------------------------------------------
// Ising and kinetic models.  The smooth part f(w) of a pair's objective
// (coupling w, the rest of W fixed) has f'(0) = a, the contraction entry
//   Ising:   a_ij = x_i . r_j + r_i . x_j   (r = x - tanh h)
//   kinetic: a_ij = r_i . x_j               (i <- j; r_i = x_{i,t} - tanh h_{i,t-1},
//                                            x_j = x_{j,t-1})
// and curvature C(w) = -f''(w) = sum over the affected samples of
// sech^2(h + w x) with x = +-1.  Since cosh h e^{-|w|} <= cosh(h + w x) <=
// cosh h e^{|w|},  c e^{-2|w|} <= C(w) <= c e^{2|w|}  with c = C(0) = sum of
// (1 - tanh^2 h) over those samples (Ising: c_i + c_j; kinetic: c_i).  For a
// pair with w0 = 0 and e = |a| - lambda > 0, integrating f' twice under these
// bounds brackets the best gain of the L1-penalised step [Alg. 2, function D]:
//   (c/4) phi(q) <= gain <= (c/4) psi(q),   q = 2e/c,
//   phi(q) = (1 + q) ln(1 + q) - q,   psi(q) = q + (1 - q) ln(1 - q)  (q < 1; else no bound),
// and gain = 0 when |a| <= lambda (the kink test).  a is formed on the int8
// matrix cores from x = +-1 and the int8 residual copies q = round(63.5 r)
// with exact int32 sums, so |a - a_exact| <= ce (E_i + E_j) + el, E_i the
// row's summed quantisation error (sum of |r - q / 63.5|).
// The two passes then run as for the Gaussian screen: a histogram of the
// lower bounds gives tau, and every w0 = 0 pair whose upper bound reaches tau
// goes to the exact score kernel together with the current couplings.  The
// result equals the exhaustive search's positive-gain top m.

struct KScreenArgs {
  const int8_t* xs;     // (N + REC_TAIL_ROWS) x Mp int8 input side (+-1; padding and tail rows 0)
  const int8_t* rq;     // (N + REC_TAIL_ROWS) x Mp int8 residuals (padding and tail rows 0)
  int64_t N, Mp;
  int opbytes;          // bytes of each operand array, (N + REC_TAIL_ROWS) Mp < 2^31
  int nsteps;           // k steps of KS_K samples: Ising 2 Mp / KS_K, kinetic Mp / KS_K
  const float* l1;      // E_i, the int8 copy's total error on row i, rounded up
  const float* cv;      // c_i = sum_t (1 - tanh^2 h_it)
  const float* cvmin;   // min_i c_i (Ising: bounds c_i + c_j from below per row)
  float lam, ce, el;
  uint32_t* hist;
  const float* tau;     // collect threshold
  const float* hfloor;  // histogram floor (null: none)
  WTable W;
  int32_t* oi;
  int32_t* oj;
  float* og;            // upper bound of each collected pair
  int32_t* ovf;         // set when a block queue overflowed (that pass is then incomplete)
  int64_t* cursor;
  int64_t cap;
  int32_t* err;
};

// per node: E_i = sum_m |r_im - q_im / 63.5|, the total error of the int8
// residual copy the contraction reads against the working-precision residual
// r = y - tanh h (rounded up), and c_i = sum_m (1 - tanh^2 h_im)
template <class R>
__global__ __launch_bounds__(256) void k_kscreen_prep(Fields F, float* __restrict__ l1,
                                                      float* __restrict__ cv) {
  __shared__ double sh[8];
  const int64_t i = blockIdx.x;
  const R* T = reinterpret_cast<const R*>(F.T) + i * F.Mp;
  const int8_t* q = F.rq + i * F.Mp;
  const int8_t* y = F.ys + i * F.Mp;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t k = threadIdx.x; k < F.M; k += blockDim.x) {
    const double t = (double)T[k];
    const double r = (double)((R)y[k] - T[k]);
    s1 += fabs(r - (double)q[k] / 63.5);
    s2 += 1.0 - t * t;
  }
  s1 = rec_wave_sum(s1);
  s2 = rec_wave_sum(s2);
  const int w = threadIdx.x / REC_WAVE;
  if ((threadIdx.x & (REC_WAVE - 1)) == 0) { sh[w] = s1; sh[4 + w] = s2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int qq = 0; qq < (int)(blockDim.x / REC_WAVE); ++qq) { a += sh[qq]; b += sh[4 + qq]; }
    l1[i] = (float)(a * (1.0 + 1e-6) + 1e-30);
    cv[i] = (float)b;
  }
}

// min_i c_i (one block)
__global__ __launch_bounds__(1024) void k_ks_cvmin(const float* __restrict__ cv, int64_t N, float* out) {
  __shared__ float sh[16];
  float v = __builtin_inff();
  for (int64_t i = threadIdx.x; i < N; i += 1024) v = fminf(v, cv[i]);
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, REC_WAVE));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = sh[0];
    for (int q = 1; q < 16; ++q) m = fminf(m, sh[q]);
    *out = m;
  }
}

// lower bound (c/4) phi(q) and upper bound (c/4) psi(q) in float with a
// relative slack that covers the float evaluation
__device__ __forceinline__ float kgain_lo(float e, float c) {
  c *= 1.f + 1e-6f;
  const float q = 2.f * e / c;
  float p;
  if (q <= 1.f)   // alternating series with decreasing terms: stop after a negative one
    p = q * q * (0.5f - q * (1.f / 6.f - q * (1.f / 12.f - q * (1.f / 20.f))));
  else
    p = (1.f + q) * log1pf(q) - q;
  return 0.25f * c * p * (1.f - 1e-5f);
}

__device__ __forceinline__ float kgain_up(float e, float c) {
  c *= 1.f - 1e-6f;
  const float q = 2.f * e / c;
  if (q >= 1.f) return __builtin_inff();
  float p;
  if (q <= 0.5f)  // positive series q^k / (k (k-1)), tail from k = 6 bounded geometrically
    p = q * q * (0.5f + q * (1.f / 6.f + q * (1.f / 12.f + q * (1.f / 20.f + q * q / (30.f * (1.f - q))))));
  else
    p = q + (1.f - q) * log1pf(-q);
  return 0.25f * c * p * (1.f + 1e-5f);
}

// LDS operand layout: rows of KS_K = 128 int8 samples (128 bytes, no
// padding); the 16-byte chunk c of row r sits at slot c ^ (r & 7).  A fragment read (rows
// 16k..16k+15 at one chunk) and a staging write (8 lanes per row) touch 8
// distinct 16-byte slots in every 8 lanes: no bank conflicts (checked with
// the LDS bank-conflict counters on gfx950, which serve ds_read_b128 in
// 8-lane groups; padded rows and XORs over wider lines conflict 2-way).
__device__ __forceinline__ int ks_swz(int r, int c) { return r * 128 + 16 * (c ^ (r & 7)); }   // bytes


// Histogram of positive float bounds for the Ising / kinetic screen: 16 bins
// per octave over [2^-31, 2^33); smaller values are not counted (a threshold
// of 0 then remains valid), larger ones land in the top bin (whose lower edge
// still bounds them from below).
constexpr int KS_BINS = 1024;
constexpr int KS_EXP0 = 96;   // biased exponent of the lowest bin
__device__ __forceinline__ int ks_bin(float g) {
  const int b = (int)(__builtin_bit_cast(uint32_t, g) >> 19) - KS_EXP0 * 16;
  return b < 0 ? -1 : (b >= KS_BINS ? KS_BINS - 1 : b);
}
__host__ __device__ inline float ks_edge(int b) {
  const uint32_t bits = (uint32_t)(b + KS_EXP0 * 16) << 19;
  float f;
  __builtin_memcpy(&f, &bits, 4);
  return f;
}

// Tile order.  Hardware hands block b to XCD b % 8; blocks that run together
// on one XCD should share their operand rows in that XCD's L2.  Logical tiles
// form super-tiles of 8 x 8 (8 row tiles x 8 column tiles: the ~64 blocks an
// XCD runs at once), super-tiles are dealt to the XCDs round-robin, and an XCD
// walks its super-tiles in order.
struct TileMap {
  int nbi, nbj;     // row tiles (after sampling) and column tiles
  int sbj;          // super-tile columns
  int nS;           // super-tiles
};
__device__ __forceinline__ bool ks_tile(const TileMap& T, int b, int* bi, int* bj) {
  const int x = b & 7, q = b >> 3;
  const int S = (q >> 6) * 8 + x, w = q & 63;
  if (S >= T.nS) return false;
  *bi = (S / T.sbj) * 8 + (w & 7);
  *bj = (S % T.sbj) * 8 + (w >> 3);
  return *bi < T.nbi && *bj < T.nbj;
}

// One KS_BM x KS_BN tile of the contraction per block (8 waves of 128 x 64,
// each 8 x 4 MFMA 16x16x64 int8 blocks with int32 accumulators: the +-1
// samples times the int8 residual copies sum exactly).  Operands go global ->
// LDS directly, one step ahead of use (LDS double-buffered), and a tile's
// first step loads during the previous tile's epilogue.  Ising: tiles that hold a
// pair i < j, k in [0, Mp) pairs x_i with r_j and k in [Mp, 2Mp) r_i with x_j.
// Kinetic: every tile, rows are targets (r_i), columns sources (x_j).
// MODE 0: histogram of lower bounds; 1: collect pairs whose upper bound
// reaches *tau; 2: both.  Row tiles are taken every row_step-th (sampling).
// Tile of the contraction: KS_THREADS / 64 wavefronts in KS_WR x KS_WC, each
// KS_WM x KS_WN blocks of 16 x 16 outputs; the block covers KS_BM rows x
// KS_BN columns.
constexpr int KS_THREADS = 512;
constexpr int KS_K = 128;  // samples (bytes) per k step (two MFMA k-substeps of 64)
constexpr int KS_WR = 2, KS_WC = 4;
constexpr int KS_WM = 8, KS_WN = 4;
constexpr int KS_BM = KS_WR * KS_WM * 16, KS_BN = KS_WC * KS_WN * 16;
constexpr int KS_Q = 2 * KS_THREADS;   // per-block queue of elements that passed the cheap tests (LDS)
constexpr int KS_OB = KS_Q;            // per-block batch of collected pairs (LDS); >= one tile's worth
static_assert(KS_WR * KS_WC * REC_WAVE == KS_THREADS, "one wavefront per sub-tile");
static_assert(KS_BM <= REC_TAIL_ROWS && KS_BN <= REC_TAIL_ROWS, "tiles must stay inside the zero tail");
static_assert(KS_BM <= 256 && KS_BN <= 256, "queue keys hold 8-bit rows and columns");
static_assert(KS_BM % (KS_THREADS / 8) == 0 && KS_BN % (KS_THREADS / 8) == 0, "staging rows per thread");

template <int MODE, int KIN, int ROBUST>
__global__ __launch_bounds__(KS_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_kscreen(KScreenArgs P, TileMap TM, int row_step, int* tctr, int nvirt) {
  constexpr bool HIST = MODE != 1, COLLECT = MODE != 0;
  // operand buffers (two steps of each operand), separate objects so that
  // reads of one need not wait on loads landing in another
  __shared__ __attribute__((aligned(16))) int8_t As0[KS_BM * KS_K], As1[KS_BM * KS_K];
  __shared__ __attribute__((aligned(16))) int8_t Bs0[KS_BN * KS_K], Bs1[KS_BN * KS_K];
  __shared__ uint32_t hs[HIST ? KS_BINS : 1];
  __shared__ uint32_t kq_key[KS_Q];   // bit 31 histogram, bit 30 collect; row << 8 | column in the tile
  __shared__ float kq_e[KS_Q];
  // the tile's raw per-row and per-column terms (|r|_1 and c), loaded with
  // the operands' first step
  __shared__ float tl1r[KS_BM], tcvr[KS_BM], tl1c[KS_BN], tcvc[KS_BN];
  __shared__ int kq_n, kc_n;
  __shared__ int64_t kbase;
  __shared__ int s_q;
  // collected pairs of this block's tiles, written out in batches (one global
  // atomic per batch instead of per tile)
  __shared__ int32_t ob_i[COLLECT ? KS_OB : 1], ob_j[COLLECT ? KS_OB : 1];
  __shared__ float ob_g[COLLECT ? KS_OB : 1];
  __shared__ int ob_n;
  const int tid = threadIdx.x, lane = tid & (REC_WAVE - 1), w = tid / REC_WAVE;
  if (HIST)
    for (int q = tid; q < KS_BINS; q += KS_THREADS) hs[q] = 0;
  // Persistent blocks (one per CU): block b takes the virtual block indices
  // of its XCD (b & 7) from that XCD's counter, i.e. the tiles the hardware
  // would have dealt to that XCD, so its L2 keeps serving its super-tiles;
  // the block's histogram is flushed once at the end.
  const int xcd = blockIdx.x & 7;
  if (tid == 0) {
    s_q = atomicAdd(&tctr[xcd], 1);
    ob_n = 0;
  }
  __syncthreads();
  // write the batch out (all threads; uniform)
  auto flush = [&]() {
    const int nb = ob_n;
    if (tid == 0) kbase = (int64_t)atomicAdd((unsigned long long*)P.cursor, (unsigned long long)nb);
    __syncthreads();
    for (int t = tid; t < nb; t += KS_THREADS) {
      const int64_t pos = kbase + t;
      if (pos < P.cap) {
        P.oi[pos] = ob_i[t];
        P.oj[pos] = ob_j[t];
        P.og[pos] = ob_g[t];
      }
    }
    __syncthreads();
    if (tid == 0) ob_n = 0;
    __syncthreads();
  };
  // Staging: operands go global -> LDS directly (buffer loads to LDS, no
  // registers): one wave instruction fills 8 rows of 128 bytes, lane l
  // moving row R + l/8 into slot l % 8, which under the swizzle holds sample
  // chunk (l % 8) ^ (l / 8) (R is a multiple of 8).  Wave w fills rows
  // 8 w + SRS u of both operands.  Operand rows are int8 (the +-1 input side
  // and the residual copies) with zero rows past N, so no load needs a bound
  // check.  Ising: in the first half of k, A = x and B = r; in the second,
  // A = r and B = x.  Kinetic: A = r (targets), B = x (sources).  Rows hold a
  // multiple of KS_K samples, so a step lies inside one half.
  constexpr int SRS = KS_THREADS / 8;   // rows per staging round (all waves)
  constexpr int NA = KS_BM / SRS, NB = KS_BN / SRS;
  static_assert(KS_THREADS / REC_WAVE >= 4 && KS_BM == 4 * REC_WAVE && KS_BN == 4 * REC_WAVE, "term loads");
  const int n = P.nsteps;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int srow = 8 * wu + (lane >> 3), schunk = (lane & 7) ^ (lane >> 3);
  const uint32_t ostep = (uint32_t)(SRS * P.Mp);   // global offset between staging rounds
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void*)P.xs, 0, P.opbytes, KS_RSRC3);
  const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc((void*)P.rq, 0, P.opbytes, KS_RSRC3);
  // the per-row terms: reads past N return 0 (range-checked buffer loads)
  const __amdgpu_buffer_rsrc_t rl1 = __builtin_amdgcn_make_buffer_rsrc((void*)P.l1, 0, (int)(P.N * 4), KS_RSRC3);
  const __amdgpu_buffer_rsrc_t rcv = __builtin_amdgcn_make_buffer_rsrc((void*)P.cv, 0, (int)(P.N * 4), KS_RSRC3);
  // step s of the tile at rows r0, columns c0 into LDS buffers A, B
  auto issue = [&](int s, int64_t r0, int64_t c0, int8_t* A, int8_t* B) {
    const bool first = !KIN && s * KS_K < P.Mp;
    const int k = s * KS_K - (KIN || first ? 0 : (int)P.Mp);
    const __amdgpu_buffer_rsrc_t ra = first ? rx : rr, rb = first ? rr : rx;
    const uint32_t oa0 = (uint32_t)((r0 + srow) * P.Mp + schunk * 16);
    const uint32_t ob0 = (uint32_t)((c0 + srow) * P.Mp + schunk * 16);
#pragma unroll
    for (int u = 0; u < NA; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (__attribute__((address_space(3))) void*)(A + (8 * wu + SRS * u) * KS_K),
                                               16, (int)(oa0 + u * ostep), k, 0, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (__attribute__((address_space(3))) void*)(B + (8 * wu + SRS * u) * KS_K),
                                               16, (int)(ob0 + u * ostep), k, 0, 0);
  };
  // the first step of a tile and its row and column terms (waves 0-3: 64
  // rows or columns of one term each)
  auto issue_tile = [&](int64_t r0, int64_t c0) {
    issue(0, r0, c0, As0, Bs0);
    if (wu < 4) {
      const __amdgpu_buffer_rsrc_t rt = (wu & 1) ? rcv : rl1;
      float* dst = wu == 0 ? tl1r : wu == 1 ? tcvr : wu == 2 ? tl1c : tcvc;
      const int64_t base = wu < 2 ? r0 : c0;
      for (int h = 0; h < 4; ++h)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rt, (__attribute__((address_space(3))) void*)(dst + h * REC_WAVE), 4,
                                                 (int)((base + h * REC_WAVE + lane) * 4), 0, 0, 0);
    }
  };
  // this wave's loads to LDS have landed (the barrier that follows makes
  // every wave's visible)
  auto landed = [&]() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); };
  // tile of virtual block index v: its rows and columns, false if it has no
  // pair to score
  auto tile_of = [&](int v, int64_t* r0, int64_t* c0) -> bool {
    int bi, bj;
    bool ok = v < nvirt && ks_tile(TM, v, &bi, &bj);
    *r0 = (int64_t)(bi * row_step) * KS_BM;
    *c0 = (int64_t)bj * KS_BN;
    if (!KIN && *r0 >= *c0 + KS_BN - 1) ok = false;   // no pair i < j in the tile
    return ok;
  };
  int tq = s_q;
  bool pre = false;   // the tile's first step was loaded during the last epilogue
  for (;;) {
  const int vb = tq * 8 + xcd;
  if (vb >= nvirt) break;
  __syncthreads();   // every thread has read s_q and is done with the last tile's LDS
  if (tid == 0) {
    s_q = atomicAdd(&tctr[xcd], 1);
    kq_n = 0;
    kc_n = 0;
  }
  int64_t r0, c0;
  const bool ok = tile_of(vb, &r0, &c0);
  if (ok) {
  intx4 iacc[KS_WM][KS_WN];
#pragma unroll
  for (int m = 0; m < KS_WM; ++m)
#pragma unroll
    for (int q = 0; q < KS_WN; ++q) iacc[m][q] = intx4{0, 0, 0, 0};
  const int wr = (w / KS_WC) * (KS_WM * 16), wc = (w % KS_WC) * (KS_WN * 16);
  // fragments of k-substep h: lane l reads row (block base + l % 16), chunk
  // 4h + l / 16
  int fa[KS_WM][2], fb[KS_WN][2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int f = 0; f < KS_WM; ++f) fa[f][h] = ks_swz(wr + f * 16 + (lane & 15), 4 * h + (lane >> 4));
#pragma unroll
    for (int f = 0; f < KS_WN; ++f) fb[f][h] = ks_swz(wc + f * 16 + (lane & 15), 4 * h + (lane >> 4));
  }
  auto compute = [&](const int8_t* A, const int8_t* B) {
    __builtin_amdgcn_iglp_opt(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      intx4 bf[KS_WN];
#pragma unroll
      for (int q = 0; q < KS_WN; ++q) bf[q] = *reinterpret_cast<const intx4*>(B + fb[q][h]);
#pragma unroll
      for (int m = 0; m < KS_WM; ++m) {
        const intx4 af = *reinterpret_cast<const intx4*>(A + fa[m][h]);
#pragma unroll
        for (int q = 0; q < KS_WN; ++q)
          iacc[m][q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[q], iacc[m][q], 0, 0, 0);
      }
    }
  };
  // Step s reads buffer s % 2 while step s + 1 lands in the other, which
  // every wave finished reading at the barrier ending step s - 1.  The loop
  // body has no branches: past the end, the last step loads again into a
  // buffer nobody reads (it lands before the barrier).
  if (!pre) issue_tile(r0, c0);
  landed();
  __syncthreads();
  for (int s = 0; s + 1 < n; s += 2) {
    issue(s + 1, r0, c0, As1, Bs1);
    compute(As0, Bs0);
    landed();
    __syncthreads();
    issue(min(s + 2, n - 1), r0, c0, As0, Bs0);
    compute(As1, Bs1);
    landed();
    __syncthreads();
  }
  // (an odd last step reads buffer 0; the epilogue's LDS lies in buffer 1)
  if (n & 1) compute(As0, Bs0);
  // a = (sum of x q) / 63.5: the int32 sums are exact and below 2^24 in
  // magnitude (127 x 2 Mp), so the float conversion is exact and the scaling
  // rounds once (2^-24 relative, inside the slack el); converted where used
#define KS_ACC(m, q, r) ((float)iacc[m][q][r] * REC_Q8_INV)
  // Epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each
  // 16x16 block.  Each element first meets per-row and per-column necessary
  // conditions (a few ALU operations); the rare survivors go to a block
  // queue in LDS and get the exact bound afterwards.  With q = 2e/c:
  // (c/4) psi(q) <= e^2 / (2 (c - 2e)), so an upper bound can reach tau only
  // if e >= sqrt(4 tau^2 + 2 tau c) - 2 tau;  (c/4) phi(q) <= e^2 / (2c), so
  // a lower bound can reach the floor f only if e >= sqrt(2 f c).  Both grow
  // with c, and c >= c_i + min c (Ising) or c = c_i (kinetic).
  // The epilogue's lane-derived indices are formed from an opaque copy of the
  // lane id, per tile: otherwise the compiler hoists them out of the tile
  // loop, and they stay live across the k loop and spill.
  int elane = lane;
  asm volatile("" : "+v"(elane));
  const float tau = COLLECT ? *P.tau : 0.f;
  const float fl = HIST && P.hfloor ? *P.hfloor : 0.f;
  const float cmin = KIN ? 0.f : *P.cvmin;
  auto thr_up = [&](float c) {
    return tau > 0.f ? (sqrtf(4.f * tau * tau + 2.f * tau * c) - 2.f * tau) * (1.f - 1e-4f) : 0.f;
  };
  auto thr_lo = [&](float c) { return fl > 0.f ? sqrtf(2.f * fl * c) * (1.f - 1e-4f) : 0.f; };
  // Per-row and per-column terms, one thread per row / column, into LDS (the
  // operand buffers are free after the k loop): row (er_i, c_i, up_i, lo_i)
  // with er_i = ce |r_i|_1 + el and up/lo the gate thresholds at c_i + min c;
  // column (ce |r_j|_1, c_j, up_j, lo_j) (Ising; zeros for kinetic).
  // Kinetic: also each row's pre-test threshold (its gate, or lambda + er_i
  // for the sampling estimate, less a float slack), so that a wave reads four
  // rows' thresholds with one load.
  float4* rowv = reinterpret_cast<float4*>(As1);
  float4* colv = rowv + KS_BM;
  float* qrow = reinterpret_cast<float*>(colv + KS_BN);
  for (int t = tid; t < KS_BM + KS_BN; t += KS_THREADS) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < KS_BM) {
      const float l1 = tl1r[t], c = tcvr[t];   // 0 past N
      v = make_float4(P.ce * l1 + P.el, c, thr_up(c + cmin), thr_lo(c + cmin));
      rowv[t] = v;
      if (KIN) {
        const float big = __builtin_inff();
        float qg = (MODE == 0 && !ROBUST)
                       ? P.lam + v.x
                       : fminf(COLLECT ? P.lam - v.x + v.z : big, HIST ? P.lam + v.x + v.w : big);
        qg -= fabsf(qg) * 1e-5f + 1e-30f;
        qrow[t] = qg;
      }
    } else if (!KIN) {
      const float l1 = tl1c[t - KS_BM], c = tcvc[t - KS_BM];   // 0 past N
      v = make_float4(P.ce * l1, c, thr_up(c + cmin), thr_lo(c + cmin));
      colv[t - KS_BM] = v;
    } else {
      colv[t - KS_BM] = v;
    }
  }
  // Ising: the column threads (whole wavefronts) reduce the tile's column
  // terms to their extremes, from which each row's pre-test threshold is
  // formed: the gate with every column term at its least favourable value.
  float4* cext = reinterpret_cast<float4*>(qrow + KS_BM);   // one entry per column wavefront
  static_assert(KS_BM % REC_WAVE == 0 && KS_THREADS - KS_BM <= 4 * REC_WAVE, "column wavefronts");
  if (!KIN && tid >= KS_BM) {
    const float4 v = colv[tid - KS_BM];
    float amax = v.x, amin = v.x, umin = v.z, hmin = v.w;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      amax = fmaxf(amax, __shfl_xor(amax, o, REC_WAVE));
      amin = fminf(amin, __shfl_xor(amin, o, REC_WAVE));
      umin = fminf(umin, __shfl_xor(umin, o, REC_WAVE));
      hmin = fminf(hmin, __shfl_xor(hmin, o, REC_WAVE));
    }
    if (lane == 0) cext[(tid - KS_BM) / REC_WAVE] = make_float4(amax, amin, umin, hmin);
  }
  __syncthreads();
  // Every thread has read the tile's terms and the operand buffers are free:
  // the next tile's first step and terms load during the rest of the
  // epilogue (s_q holds the next virtual block since the barrier after its
  // atomic).
  {
    int64_t r0n, c0n;
    pre = tile_of(s_q * 8 + xcd, &r0n, &c0n);
    if (pre) issue_tile(r0n, c0n);
  }
  if (!KIN) {
    if (tid < KS_BM) {
      float amax = cext[0].x, amin = cext[0].y, umin = cext[0].z, hmin = cext[0].w;
#pragma unroll
      for (int c = 1; c < (KS_THREADS - KS_BM) / REC_WAVE; ++c) {
        amax = fmaxf(amax, cext[c].x);
        amin = fminf(amin, cext[c].y);
        umin = fminf(umin, cext[c].z);
        hmin = fminf(hmin, cext[c].w);
      }
      const float4 v = rowv[tid];
      const float big = __builtin_inff();
      float qg = (MODE == 0 && !ROBUST)
                     ? P.lam + v.x + amin
                     : fminf(COLLECT ? P.lam - v.x - amax + fmaxf(v.z, umin) : big,
                             HIST ? P.lam + v.x + amin + fmaxf(v.w, hmin) : big);
      qg -= fabsf(qg) * 1e-5f + 1e-30f;
      qrow[tid] = qg;
    }
    __syncthreads();
  }
  float cl1[KS_WN], ccv[KS_WN], cu[KS_WN], ch[KS_WN];
#pragma unroll
  for (int q = 0; q < KS_WN; ++q) {
    const float4 v = colv[wc + q * 16 + (elane & 15)];
    cl1[q] = v.x;
    ccv[q] = v.y;
    cu[q] = v.z;
    ch[q] = v.w;
  }
  // Every element that passes its gate and the range/threshold checks
  // enters the block queue (key: bit 31 histogram, bit 30 collect, row << 8 |
  // column; then |a|; c comes from the row and column terms), which is then
  // settled.  ROBUST: once the queue
  // is full the rest wait for the next round (done bits: element (m, r, q) is
  // bit (m*4 + r)*KS_WN + q) until a round fits; otherwise one round, and an
  // overflow is flagged for the caller.  MODE 0 without ROBUST is the
  // sampling estimate and histograms inline.
  uint32_t done[KS_WM * 4 * KS_WN / 32];
#pragma unroll
  for (int d = 0; d < KS_WM * 4 * KS_WN / 32; ++d) done[d] = 0u;
  for (;;) {
    // One gate per element: |a| must reach lambda - er + the collect
    // threshold or lambda + er + the histogram threshold (kinetic: one value
    // per row).  Range and triangle checks run only behind the gate (padding
    // rows and columns hold a = 0).
#pragma unroll
    for (int m = 0; m < KS_WM; ++m) {
      const float4 q4 = *reinterpret_cast<const float4*>(&qrow[wr + m * 16 + 4 * (elane >> 4)]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = wr + m * 16 + 4 * (elane >> 4) + r;
        const int64_t i = r0 + li;
        {   // row pre-test from the stored threshold (see below)
          float mx = fabsf(KS_ACC(m, 0, r));
#pragma unroll
          for (int q = 1; q < KS_WN; ++q) mx = fmaxf(mx, fabsf(KS_ACC(m, q, r)));
          const float qg = r == 0 ? q4.x : r == 1 ? q4.y : r == 2 ? q4.z : q4.w;
          if (__ballot(mx >= qg) == 0) continue;
        }
        const float4 rv = rowv[li];
        const float er_row = rv.x, rcv = rv.y, ru = rv.z, rh = rv.w;
        const float big = __builtin_inff();
        const float gate_row = fminf(COLLECT ? P.lam - er_row + ru : big, HIST ? P.lam + er_row + rh : big);
        // (Row pre-test above: the largest |a| of the lane's entries in this
        // row against a lower bound of their gates, stored per row: kinetic,
        // the row gate; Ising, the gate with the column terms at their extremes
        // over the tile; sampling, lambda + the smallest error bound; less a
        // float slack.  A row that no lane passes is skipped by the whole
        // wave, so the per-element tests run only on rows holding candidates.)
#pragma unroll
        for (int q = 0; q < KS_WN; ++q) {
          const int bit = (m * 4 + r) * KS_WN + q;
          const float aa = fabsf(KS_ACC(m, q, r));
          if (MODE == 0 && !ROBUST) {
            // sampling estimate: histogram e^2 / (2c) (the quadratic model of
            // the gain) inline, no queue
            const float er = er_row + cl1[q];
            const float e = aa - er - P.lam;
            if (e > 0.f) {
              const int lj = wc + q * 16 + (elane & 15);
              const int64_t j = c0 + lj;
              const bool ok = KIN ? (i < P.N && j < P.N && i != j) : (i < j && j < P.N);
              const int hb = ks_bin(e * e / (2.f * (rcv + ccv[q])));
              if (ok && hb >= 0) atomicAdd(&hs[hb], 1u);
            }
            continue;
          }
          float gate = gate_row;
          if (!KIN) {
            const float er = er_row + cl1[q];
            gate = fminf(COLLECT ? P.lam - er + fmaxf(ru, cu[q]) : big,
                         HIST ? P.lam + er + fmaxf(rh, ch[q]) : big);
          }
          if (aa >= gate && !((done[bit >> 5] >> (bit & 31)) & 1u)) {
            const int lj = wc + q * 16 + (elane & 15);
            const int64_t j = c0 + lj;
            const bool ok = KIN ? (i < P.N && j < P.N && i != j) : (i < j && j < P.N);
            const float er = er_row + cl1[q];
            const float el = aa - er - P.lam, eu = aa + er - P.lam;
            const bool h = HIST && ok && el > 0.f && el >= rh && el >= ch[q];
            const bool cc = COLLECT && ok && eu > 0.f && eu >= ru && eu >= cu[q];
            bool fin = true;
            if (h || cc) {
              const int p = atomicAdd(&kq_n, 1);
              if (p < KS_Q) {
                kq_key[p] = (h ? 0x80000000u : 0u) | (cc ? 0x40000000u : 0u) | (uint32_t)li << 8 | (uint32_t)lj;
                kq_e[p] = aa;
              } else {
                fin = false;
              }
            }
            if (fin) done[bit >> 5] |= 1u << (bit & 31);
          }
        }
      }
    }
    __syncthreads();
    if (MODE == 0 && !ROBUST) break;
    const int nq = min(kq_n, KS_Q);
    const bool more = kq_n > KS_Q;
    if (!ROBUST && more && tid == 0) atomicOr(P.ovf, 1);   // the caller falls back to the robust pass
    // settle: exact bounds; collected pairs are compacted into the queue's
    // front (every slot of the round is read before the sync, written after)
    uint32_t key[2] = {0u, 0u};
    float av[2] = {0.f, 0.f}, cv2[2] = {0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = u * KS_THREADS + tid;
      if (t < nq) {
        key[u] = kq_key[t];
        av[u] = kq_e[t];
        cv2[u] = rowv[(key[u] >> 8) & 255].y + colv[key[u] & 255].y;   // c of the pair, as the gate formed it
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = u * KS_THREADS + tid;
      if (t >= nq) continue;
      const int li = (int)((key[u] >> 8) & 255), lj = (int)(key[u] & 255);
      // the error bound from the tile's row and column terms in LDS (the sum
      // the gates used), not from global memory
      const float er = rowv[li].x + colv[lj].x;
      if (HIST && (key[u] >> 31)) {
        const int hb = ks_bin(kgain_lo(av[u] - er - P.lam, cv2[u]));
        if (hb >= 0) atomicAdd(&hs[hb], 1u);
      }
      if (COLLECT && ((key[u] >> 30) & 1u)) {
        const float gu = kgain_up(av[u] + er - P.lam, cv2[u]);
        // (a current coupling collected here is dropped by the filter pass,
        // which looks the pairs up in W off this kernel's critical path)
        const bool keep = gu >= tau;
        if (keep) {
          const int pc = atomicAdd(&kc_n, 1);   // pc < KS_Q: at most one per queued element
          kq_key[pc] = (uint32_t)li << 8 | (uint32_t)lj;
          kq_e[pc] = gu;
        }
      }
    }
    if (COLLECT) {
      __syncthreads();
      const int nc = kc_n;
      if (ob_n + nc > KS_OB) flush();
      const int base = ob_n;
      for (int t = tid; t < nc; t += KS_THREADS) {
        ob_i[base + t] = (int32_t)(r0 + ((kq_key[t] >> 8) & 255));
        ob_j[base + t] = (int32_t)(c0 + (kq_key[t] & 255));
        ob_g[base + t] = kq_e[t];
      }
      __syncthreads();
      if (tid == 0) ob_n = base + nc;
    }
    __syncthreads();
    if (!ROBUST || !more) break;
    if (tid == 0) { kq_n = 0; kc_n = 0; }
    __syncthreads();
  }
  } else {
    pre = false;
  }   // tile
  __syncthreads();
  tq = s_q;
  }   // tiles of this block
  if (COLLECT && ob_n > 0) flush();
  if (HIST)
    for (int q = tid; q < KS_BINS; q += KS_THREADS)
      if (hs[q]) atomicAdd(&P.hist[q], hs[q]);
}
#undef KS_ACC

// Current couplings (w0 != 0), first pass, before the full pass's threshold
// is taken: one wavefront per coupling forms a, the gradient at the current
// state, from the int8 rows (error bounded as for the contraction) and keeps
// it in wa.  The contraction histograms every pair as if it were new,
// couplings included; here each coupling adds one count in the bin of an
// upper bound on the value the contraction could have binned for it (a off
// by at most er on each side, 0.1% slack for the float evaluation), so that
// the full histogram minus these counts bounds from below, over every bin
// edge, the number of new pairs (w0 = 0) whose lower bound reaches it.
constexpr int KS_CA_PER_BLOCK = 64;   // couplings per block of k_ks_couple_a
template <int KIN>
__global__ __launch_bounds__(256) void k_ks_couple_a(KScreenArgs P, const int32_t* __restrict__ wi,
                                                     const int32_t* __restrict__ wj, int64_t nnz,
                                                     float* __restrict__ wa, uint32_t* __restrict__ hist_c) {
  // the block's counts gather in LDS first: couplings near their optimum
  // crowd a few bins, which would serialise global atomics
  __shared__ uint32_t hb_s[KS_BINS];
  for (int q = threadIdx.x; q < KS_BINS; q += 256) hb_s[q] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & (REC_WAVE - 1);
  const int64_t e_end = min(nnz, ((int64_t)blockIdx.x + 1) * KS_CA_PER_BLOCK);
  for (int64_t e = (int64_t)blockIdx.x * KS_CA_PER_BLOCK + (threadIdx.x / REC_WAVE); e < e_end; e += 4) {
    const int64_t i = wi[e], j = wj[e];
    const int8_t* ri = P.rq + i * P.Mp;
    const int8_t* xj = P.xs + j * P.Mp;
    const int8_t* rj = P.rq + j * P.Mp;
    const int8_t* xi = P.xs + i * P.Mp;
    int isum = 0;   // exact: |sum| <= 127 x 2 Mp
    for (int64_t k = (int64_t)lane * 16; k < P.Mp; k += 16 * REC_WAVE) {
      const intx4 a = *reinterpret_cast<const intx4*>(ri + k);
      const intx4 b = *reinterpret_cast<const intx4*>(xj + k);
#pragma unroll
      for (int q = 0; q < 4; ++q) isum = __builtin_amdgcn_sdot4(a[q], b[q], isum, false);
      if (!KIN) {
        const intx4 c = *reinterpret_cast<const intx4*>(rj + k);
        const intx4 d = *reinterpret_cast<const intx4*>(xi + k);
#pragma unroll
        for (int q = 0; q < 4; ++q) isum = __builtin_amdgcn_sdot4(c[q], d[q], isum, false);
      }
    }
    const float acc = (float)rec_wave_sum(isum) * REC_Q8_INV;
    if (lane == 0) {
      wa[e] = acc;
      const float er = P.ce * (P.l1[i] + (KIN ? 0.f : P.l1[j])) + P.el;
      const float c = P.cv[i] + (KIN ? 0.f : P.cv[j]);
      const float eu = fabsf(acc) + er - P.lam;
      if (eu > 0.f) {
        const int hb = ks_bin(kgain_lo(eu, c) * 1.001f);
        if (hb >= 0) atomicAdd(&hb_s[hb], 1u);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < KS_BINS; q += 256)
    if (hb_s[q]) atomicAdd(&hist_c[q], hb_s[q]);
}

// Current couplings, second pass.  With s = sign(w0), |w0 + d| - |w0| >= s d
// for every step d, so the gain is at most the best gain of the smooth
// concave g(d) = f(w0 + d) - f(w0) - lambda s d, whose slope at 0 is
// a - lambda s and whose curvature obeys the same bounds as for a new pair:
// gain <= (c/4) psi(2 |a - lambda s| / c).  Couplings whose bound reaches
// *tau are appended after the collected candidates.
template <int KIN>
__global__ __launch_bounds__(256) void k_ks_couple(KScreenArgs P, const int32_t* __restrict__ wi,
                                                   const int32_t* __restrict__ wj,
                                                   const double* __restrict__ wv,
                                                   const float* __restrict__ wa, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool keep = false;
  int32_t i = 0, j = 0;
  if (e < nnz) {
    i = wi[e];
    j = wj[e];
    const float sgn = wv[e] > 0.0 ? 1.f : -1.f;
    const float er = P.ce * (P.l1[i] + (KIN ? 0.f : P.l1[j])) + P.el;
    const float c = P.cv[i] + (KIN ? 0.f : P.cv[j]);
    keep = kgain_up(fabsf(wa[e] - sgn * P.lam) + er, c) >= *P.tau;
  }
  const int64_t pos = rec_append(P.cursor, keep);
  if (keep && pos < P.cap) {
    P.oi[pos] = i;
    P.oj[pos] = j;
  }
}

// Keep the collected pairs whose upper bound reaches *tau (the proven
// threshold, at least the one they were collected at) and that are not
// current couplings, compacted from the front; the count goes to *cursor.
__global__ __launch_bounds__(256) void k_ks_filter(const int32_t* __restrict__ I, const int32_t* __restrict__ J,
                                                   const float* __restrict__ g, int64_t n, const float* tau,
                                                   WTable W, int directed,
                                                   int32_t* __restrict__ oI, int32_t* __restrict__ oJ,
                                                   int64_t* cursor) {
  __shared__ long long sh[256 / REC_WAVE + 1];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool keep = e < n && g[e] >= *tau;
  if (keep && W.keys != nullptr) {
    // a current (nonzero) coupling is screened with the W list instead
    const int64_t ws = rec_hash_find(W.keys, W.mask, rec_pair_key(I[e], J[e], directed != 0), REC_MAX_PROBE);
    if (ws >= 0 && W.vals[ws] != 0.0) keep = false;
  }
  const int64_t p = rec_block_append<256 / REC_WAVE>(cursor, keep, sh);
  if (p >= 0) {
    oI[p] = I[e];
    oJ[p] = J[e];
  }
}

// tau = lower edge of the bin where the count from the top (of hist, minus
// sub when given) first reaches target (0 if it never does).  out[0] = tau.
// floor_out (optional) = tau, the histogram floor of the full pass: bins at
// or above it are counted exactly, so a proven threshold at or above the
// collect threshold is found whenever one exists.
__global__ void k_ks_tau(const uint32_t* hist, const uint32_t* sub, int64_t target, float* out,
                         float* floor_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t cum = 0;
  float t = 0.f;
  for (int q = KS_BINS - 1; q >= 0; --q) {
    cum += (int64_t)hist[q] - (sub ? (int64_t)sub[q] : 0);
    if (cum >= target) { t = ks_edge(q); break; }
  }
  *out = t;
  if (floor_out) *floor_out = t;
}

}  // namespace

namespace {
// Ising / kinetic.  A sample of the row tiles (every step-th, step up to
// KS_SAMPLE) is histogrammed first for an estimate tau_s of the threshold,
// taken at twice the proportional count so that it errs low; one full pass
// then histograms the lower bounds from tau_s up and collects at tau_s.  When
// the full histogram's threshold tau (a proven lower bound on the m-th best
// gain) is at least tau_s, every pair whose upper bound reaches tau was
// collected, so the set is complete; otherwise, or when a buffer overflowed,
// a collect pass at tau runs.
constexpr int KS_SAMPLE = 32;   // largest sampling step of the row tiles

#define REC_TRY_ST(...)                      \
  do {                                       \
    rec_status st_ = (__VA_ARGS__);          \
    if (st_ != REC_OK) return st_;           \
  } while (0)

TileMap tile_map(int nbi, int nbj, int64_t* grid) {
  TileMap T;
  T.nbi = nbi;
  T.nbj = nbj;
  T.sbj = (nbj + 7) / 8;
  const int sbi = (nbi + 7) / 8;
  T.nS = sbi * T.sbj;
  *grid = (int64_t)((T.nS + 7) / 8) * 8 * 64;
  return T;
}

// Instrumentation: bracket a contraction pass with events (kind 0: full
// pass with its algorithmic flops, 1: sample pass) when timing is on.
rec_status ev_begin(rec_ctx* ctx) {
  if (!ctx->timing) return REC_OK;
  if (ctx->sev_used == 64) {
    rec_status st = rec_screen_resolve(ctx);
    if (st != REC_OK) return st;
  }
  if (ctx->sev_used == ctx->sev.size()) {
    rec_ctx::ScrEv e{};
    REC_HIP(hipEventCreate(&e.a));
    REC_HIP(hipEventCreate(&e.b));
    ctx->sev.push_back(e);
  }
  REC_HIP(hipEventRecord(ctx->sev[ctx->sev_used].a, ctx->stream));
  return REC_OK;
}
rec_status ev_end(rec_ctx* ctx, int kind, double flops) {
  if (!ctx->timing) return REC_OK;
  rec_ctx::ScrEv& e = ctx->sev[ctx->sev_used++];
  e.kind = kind;
  e.flops = flops;
  REC_HIP(hipEventRecord(e.b, ctx->stream));
  return REC_OK;
}

template <int MODE, int ROBUST>
rec_status launch_ks(rec_ctx* ctx, const KScreenArgs& P, int nbi, int nbj, int row_step) {
  int64_t grid = 0;
  const TileMap T = tile_map(nbi, nbj, &grid);
  // persistent grid: one block per CU (a multiple of 8, one share per XCD)
  int dev = 0, ncu = 0;
  REC_HIP(hipGetDevice(&dev));
  REC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t pgrid = std::min<int64_t>(grid, std::max(8, ncu / 8 * 8));
  int* tctr = reinterpret_cast<int*>(ctx->sc_tau + 16);
  REC_HIP(hipMemsetAsync(tctr, 0, 8 * sizeof(int), ctx->stream));
  // algorithmic work of a full pass: one M-term dot product (2 flops a term)
  // per ordered pair (kinetic) or two per unordered pair (Ising)
  const double N = (double)ctx->cfg.N;
  const double flops = 2.0 * N * (N - 1.0) * (double)ctx->cfg.M;
  rec_status st = ev_begin(ctx);
  if (st != REC_OK) return st;
  if (ctx->cfg.model == REC_KINETIC)
    hipLaunchKernelGGL((k_kscreen<MODE, 1, ROBUST>), dim3((unsigned)pgrid), dim3(KS_THREADS), 0, ctx->stream, P, T,
                       row_step, tctr, (int)grid);
  else
    hipLaunchKernelGGL((k_kscreen<MODE, 0, ROBUST>), dim3((unsigned)pgrid), dim3(KS_THREADS), 0, ctx->stream, P, T,
                       row_step, tctr, (int)grid);
  return ev_end(ctx, row_step == 1 ? 0 : 1, row_step == 1 ? flops : 0.0);
}

KScreenArgs ks_args(rec_ctx* ctx) {
  const int kin = ctx->cfg.model == REC_KINETIC;
  KScreenArgs P;
  P.xs = ctx->F.xs;
  P.rq = ctx->F.rq;
  P.opbytes = (int)((ctx->cfg.N + REC_TAIL_ROWS) * ctx->F.Mp);
  P.N = ctx->cfg.N;
  P.Mp = ctx->F.Mp;
  const int64_t K = kin ? ctx->F.Mp : 2 * ctx->F.Mp;
  P.nsteps = (int)(K / KS_K);
  P.l1 = ctx->sc_l1;
  P.cv = ctx->sc_cv;
  P.cvmin = ctx->sc_tau + 3;
  P.lam = (float)ctx->cfg.lambda;
  // The int8 copies' error on a pair is at most E_i (+ E_j for the Ising
  // model), the per-row sums in l1 (rounded up); the int32 sums are exact.
  P.ce = 1.0f + 1e-6f;
  // lambda's float rounding, the one rounding of the scaled sum (2^-24 of at
  // most 2 K), the exact kernel's own float rounding (K 2^-24)
  P.el = (float)(1e-6 * ctx->cfg.lambda + (double)K * std::ldexp(1.0, -22) + 1e-30);
  P.W = ctx->W;
  P.oi = ctx->ts_i;
  P.oj = ctx->ts_j;
  P.og = reinterpret_cast<float*>(ctx->cand_slot);
  P.cursor = ctx->counter + 12;
  P.cap = ctx->cand_cap;
  P.err = ctx->err_flag;
  P.tau = ctx->sc_tau;
  P.hfloor = nullptr;
  P.hist = nullptr;
  P.ovf = reinterpret_cast<int32_t*>(ctx->sc_tau + 4);
  return P;
}

rec_status kscreen_candidates(rec_ctx* ctx, int64_t m, int64_t nnz, int64_t* n_out) {
  hipStream_t s = ctx->stream;
  const int64_t N = ctx->cfg.N;
  const int kin = ctx->cfg.model == REC_KINETIC;
  if (ctx->sc_l1 == nullptr || ctx->F.rq == nullptr) { ctx->err = "screen buffers missing"; return REC_E_INVAL; }
  float* tau_c = ctx->sc_tau;       // threshold the collect pass uses
  float* tau_f = ctx->sc_tau + 1;   // proven threshold from the full histogram
  float* floor = ctx->sc_tau + 2;   // histogram floor of the full pass
  float* cvmin = ctx->sc_tau + 3;
  if (ctx->fp32)
    hipLaunchKernelGGL(k_kscreen_prep<float>, dim3(N), dim3(256), 0, s, ctx->F, ctx->sc_l1, ctx->sc_cv);
  else
    hipLaunchKernelGGL(k_kscreen_prep<double>, dim3(N), dim3(256), 0, s, ctx->F, ctx->sc_l1, ctx->sc_cv);
  hipLaunchKernelGGL(k_ks_cvmin, dim3(1), dim3(1024), 0, s, ctx->sc_cv, N, cvmin);
  KScreenArgs P = ks_args(ctx);
  const int nb = (int)((N + KS_BM - 1) / KS_BM);     // row tiles
  const int nbc = (int)((N + KS_BN - 1) / KS_BN);    // column tiles
  uint32_t* hist_s = ctx->sc_hist;
  uint32_t* hist_f = ctx->sc_hist + KS_BINS;
  uint32_t* hist_c = ctx->sc_hist + 2 * KS_BINS;   // current couplings' share of hist_f
  REC_HIP(hipMemsetAsync(ctx->sc_hist, 0, 3 * KS_BINS * sizeof(uint32_t), s));
  REC_HIP(hipMemsetAsync(P.cursor, 0, sizeof(int64_t), s));
  REC_HIP(hipMemsetAsync(P.ovf, 0, sizeof(int32_t), s));
  // sample: every step-th row tile, histogram of the quadratic gain model
  // (it counts the couplings too: the estimate keeps room for all of them)
  const int step = std::max(1, std::min(KS_SAMPLE, nb / 8));
  const int nbs = (nb + step - 1) / step;
  P.hist = hist_s;
  REC_TRY_ST(launch_ks<0, 0>(ctx, P, nbs, nbc, step));
  const int64_t ts = std::max<int64_t>(1, 2 * (m + nnz) / step);
  hipLaunchKernelGGL(k_ks_tau, dim3(1), dim3(64), 0, s, hist_s, (const uint32_t*)nullptr, ts, tau_c, floor);
  // the couplings' gradients and their upper bins
  if (nnz > 0) {
    const unsigned grid = (unsigned)((nnz + KS_CA_PER_BLOCK - 1) / KS_CA_PER_BLOCK);
    if (kin)
      hipLaunchKernelGGL(k_ks_couple_a<1>, dim3(grid), dim3(256), 0, s, P, ctx->wi, ctx->wj, nnz, ctx->sc_wa, hist_c);
    else
      hipLaunchKernelGGL(k_ks_couple_a<0>, dim3(grid), dim3(256), 0, s, P, ctx->wi, ctx->wj, nnz, ctx->sc_wa, hist_c);
  }
  // full pass: histogram from the floor up, collect at tau_c; the proven
  // threshold counts m new pairs
  P.hist = hist_f;
  P.hfloor = floor;
  REC_TRY_ST(launch_ks<2, 0>(ctx, P, nb, nbc, 1));
  hipLaunchKernelGGL(k_ks_tau, dim3(1), dim3(64), 0, s, hist_f, hist_c, m, tau_f, (float*)nullptr);
  REC_HIP(hipGetLastError());
  int64_t n = 0;
  float tau[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  REC_HIP(hipMemcpyAsync(tau, ctx->sc_tau, 5 * sizeof(float), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  int32_t over = 0;
  memcpy(&over, &tau[4], sizeof(int32_t));
  // The collected set is complete when the proven threshold is at least the
  // one used and no block queue overflowed.  Otherwise collect again at the
  // proven threshold with the robust kernel, first refreshing the histogram
  // without a floor when the threshold fell below the floor (the counts
  // under it are partial) or a queue overflowed (counts were dropped).
  if (over || n > ctx->cand_cap || tau[1] < tau[0]) {
    if (over || tau[1] < tau[2]) {
      REC_HIP(hipMemsetAsync(hist_f, 0, KS_BINS * sizeof(uint32_t), s));
      P.hfloor = nullptr;
      REC_TRY_ST(launch_ks<0, 1>(ctx, P, nb, nbc, 1));
      hipLaunchKernelGGL(k_ks_tau, dim3(1), dim3(64), 0, s, hist_f, hist_c, m, tau_f, (float*)nullptr);
    }
    REC_HIP(hipMemcpyAsync(tau_c, tau_f, sizeof(float), hipMemcpyDeviceToDevice, s));
    REC_HIP(hipMemsetAsync(P.cursor, 0, sizeof(int64_t), s));
    REC_TRY_ST(launch_ks<1, 1>(ctx, P, nb, nbc, 1));
    REC_HIP(hipGetLastError());
    REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    REC_HIP(hipStreamSynchronize(s));
    ctx->sc_stat[8] += 1;
  }
  if (n > ctx->cand_cap) { ctx->err = "screen candidates exceed the candidate buffer"; return REC_E_NOMEM; }
  // keep the candidates whose bound reaches the proven threshold
  if (n > 0) {
    REC_HIP(hipMemsetAsync(P.cursor, 0, sizeof(int64_t), s));
    hipLaunchKernelGGL(k_ks_filter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctx->ts_i, ctx->ts_j,
                       P.og, n, tau_f, ctx->W, kin, ctx->cand_gi, ctx->cand_v, P.cursor);
    REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    REC_HIP(hipStreamSynchronize(s));
    REC_HIP(hipMemcpyAsync(ctx->ts_i, ctx->cand_gi, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    REC_HIP(hipMemcpyAsync(ctx->ts_j, ctx->cand_v, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  ctx->sc_stat[5] += 1;
  ctx->sc_stat[6] += kin ? (double)N * (double)(N - 1) : 0.5 * (double)N * (double)(N - 1);
  *n_out = n;
  return REC_OK;
}
}  // namespace

rec_status rec_screen_couplings(rec_ctx* ctx, int64_t nnz, int64_t* n_out) {
  hipStream_t s = ctx->stream;
  KScreenArgs P = ks_args(ctx);
  P.tau = ctx->sc_tau + 1;   // the proven threshold
  if (nnz > 0) {
    const unsigned grid = (unsigned)((nnz + 255) / 256);
    if (ctx->cfg.model == REC_KINETIC)
      hipLaunchKernelGGL(k_ks_couple<1>, dim3(grid), dim3(256), 0, s, P, ctx->wi, ctx->wj, ctx->wv, ctx->sc_wa, nnz);
    else
      hipLaunchKernelGGL(k_ks_couple<0>, dim3(grid), dim3(256), 0, s, P, ctx->wi, ctx->wj, ctx->wv, ctx->sc_wa, nnz);
    REC_HIP(hipGetLastError());
  }
  int64_t n = 0;
  REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  if (n > ctx->cand_cap) { ctx->err = "screen candidates exceed the candidate buffer"; return REC_E_NOMEM; }
  *n_out = n;
  return REC_OK;
}

rec_status rec_screen_resolve(rec_ctx* ctx) {
  for (size_t k = 0; k < ctx->sev_used; ++k) {
    rec_ctx::ScrEv& e = ctx->sev[k];
    REC_HIP(hipEventSynchronize(e.b));
    float ms = 0.f;
    REC_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    ctx->sc_stat[e.kind == 0 ? 0 : 3] += ms;
    ctx->sc_stat[e.kind == 0 ? 1 : 4] += 1;
    ctx->sc_stat[2] += e.flops;
  }
  ctx->sev_used = 0;
  return REC_OK;
}

rec_status rec_screen_candidates(rec_ctx* ctx, int64_t m, int64_t nnz, int64_t* n_out) {
  hipStream_t s = ctx->stream;
  const int64_t N = ctx->cfg.N;
  const int Kp = ctx->sc_kp;
  if (ctx->cfg.model != REC_GAUSS) return kscreen_candidates(ctx, m, nnz, n_out);
  // every current coupling is rescored; the threshold leaves room for all of them
  const int64_t target = m + nnz;
  if (ctx->sc_a == nullptr) { ctx->err = "screen buffers missing"; return REC_E_INVAL; }
  if (ctx->fp32)
    hipLaunchKernelGGL(k_screen_prep<float>, dim3(N), dim3(256), 0, s, ctx->F, Kp, ctx->sc_a, ctx->sc_b,
                       ctx->sc_nrm, ctx->sc_th2, ctx->sc_sq);
  else
    hipLaunchKernelGGL(k_screen_prep<double>, dim3(N), dim3(256), 0, s, ctx->F, Kp, ctx->sc_a, ctx->sc_b,
                       ctx->sc_nrm, ctx->sc_th2, ctx->sc_sq);
  ScreenArgs P;
  P.A = ctx->sc_a;
  P.B = ctx->sc_b;
  P.N = N;
  P.Kp = Kp;
  P.nrm = ctx->sc_nrm;
  P.th2 = ctx->sc_th2;
  P.sqf = ctx->sc_sq;
  P.lam = (float)ctx->cfg.lambda;
  P.cerr = (float)(std::ldexp(1.0, -7) + std::ldexp(1.0, -15) + (double)Kp * std::ldexp(1.0, -23) + 1e-5);
  P.elam = (float)(1e-6 * ctx->cfg.lambda + 1e-30);
  P.hist = ctx->sc_hist;
  P.tau = ctx->sc_tau;
  P.W = ctx->W;
  P.oi = ctx->ts_i;
  P.oj = ctx->ts_j;
  P.cursor = ctx->counter + 12;
  P.cap = ctx->cand_cap;
  P.err = ctx->err_flag;
  const int nb = (int)((N + SC_T - 1) / SC_T);
  REC_HIP(hipMemsetAsync(ctx->sc_hist, 0, SC_BINS * sizeof(uint32_t), s));
  REC_HIP(hipMemsetAsync(P.cursor, 0, sizeof(int64_t), s));
  const double flops = 2.0 * (double)N * (double)(N - 1) * (double)ctx->cfg.M;
  REC_TRY_ST(ev_begin(ctx));
  hipLaunchKernelGGL(k_screen<0>, dim3(nb, nb), dim3(256), 0, s, P);
  REC_TRY_ST(ev_end(ctx, 0, flops));
  hipLaunchKernelGGL(k_screen_tau, dim3(1), dim3(64), 0, s, ctx->sc_hist, target, ctx->sc_tau);
  REC_TRY_ST(ev_begin(ctx));
  hipLaunchKernelGGL(k_screen<1>, dim3(nb, nb), dim3(256), 0, s, P);
  REC_TRY_ST(ev_end(ctx, 0, flops));
  REC_HIP(hipGetLastError());
  int64_t n = 0;
  REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  if (n > ctx->cand_cap) { ctx->err = "screen candidates exceed the candidate buffer"; return REC_E_NOMEM; }
  ctx->sc_stat[5] += 1;
  ctx->sc_stat[6] += 0.5 * (double)N * (double)(N - 1);
  *n_out = n;
  return REC_OK;
}
