// Exhaustive screening contraction on the matrix cores (Gaussian model).
//
// For every pair at once, a_ij = x_i . r_j + r_i . x_j is one entry of
// S = A B^T with A_i = [x_i | r_i] and B_j = [r_j | x_j] (K = 2M, padded to a
// multiple of 32 with zeros), r the residuals of the Gaussian pseudolikelihood
// [App. A].  The closed-form gain of a pair at w0 = 0 is
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
#include <math.h>

#include "common.hpp"
#include "ctx.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

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
  for (int k0 = 0; k0 < P.Kp; k0 += SC_K) {
    // 128 rows x 32 bf16 per matrix = 512 chunks of 16 bytes; two per thread
#pragma unroll
    for (int q = tid; q < 512; q += 256) {
      const int row = q >> 2, ch = q & 3;
      const int64_t ga = r0 + row, gb = c0 + row;
      uint4 va = make_uint4(0u, 0u, 0u, 0u), vb = make_uint4(0u, 0u, 0u, 0u);
      if (ga < P.N) va = *reinterpret_cast<const uint4*>(P.A + ga * P.Kp + k0 + ch * 8);
      if (gb < P.N) vb = *reinterpret_cast<const uint4*>(P.B + gb * P.Kp + k0 + ch * 8);
      *reinterpret_cast<uint4*>(As + row * SC_LD + ch * 8) = va;
      *reinterpret_cast<uint4*>(Bs + row * SC_LD + ch * 8) = vb;
    }
    __syncthreads();
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
        } else {
          bool keep = gup > 0.f && gup >= tau;
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

}  // namespace

rec_status rec_screen_candidates(rec_ctx* ctx, int64_t target, int64_t* n_out) {
  hipStream_t s = ctx->stream;
  const int64_t N = ctx->cfg.N;
  const int Kp = ctx->sc_kp;
  if (ctx->sc_a == nullptr) { ctx->err = "the screening contraction needs the Gaussian model"; return REC_E_INVAL; }
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
  hipLaunchKernelGGL(k_screen<0>, dim3(nb, nb), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_screen_tau, dim3(1), dim3(64), 0, s, ctx->sc_hist, target, ctx->sc_tau);
  hipLaunchKernelGGL(k_screen<1>, dim3(nb, nb), dim3(256), 0, s, P);
  REC_HIP(hipGetLastError());
  int64_t n = 0;
  REC_HIP(hipMemcpyAsync(&n, P.cursor, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  if (n > ctx->cand_cap) { ctx->err = "screen candidates exceed the candidate buffer"; return REC_E_NOMEM; }
  *n_out = n;
  return REC_OK;
}
