// Learned proposal for the second-neighbour search: per-node sketches, a
// 3-layer ranking MLP run on the matrix cores, and its training kernels.
//
// The proposal is not part of the paper.  It ranks the candidate pairs of an
// NNDescent iteration [Alg. 4] so that only the most promising fraction gets
// the exact score d(i, j) [Alg. 2, function D]; the exact score stays the
// judge of every pair that enters a list.  Definitions:
//
// * Sketch of node i (64 floats).  x_i input-side samples, y_i targets (Ising:
//   y = x; kinetic: x_{i,t+1}; Gaussian: y = x), t_i = tanh h_i, r_i = y_i - t_i
//   (Gaussian: r_i = the residual, t_i := r_i), P in {+-1}^{28 x M} with
//   P[d][m] = -1 iff the top bit of ctr(seed, 7, d, m) is set:
//     s[0:28] = P (x + r) / sqrt(M),  s[28:56] = P (x - r) / sqrt(M),
//     s[56:64] = mean y, mean t, var t, mean |h| (Gaussian: mean |r|),
//                mean r^2, log(1 + deg), sum_j |W_ij|, theta.
//   E[P^T P] = 28 I, so sum_d s_i[d] s_j[d] - s_i[28+d] s_j[28+d] estimates
//   (56 / M)(x_i . r_j + r_i . x_j), the pair's kink-test value Phi(0).
// * Pair feature phi = [s_i * s_j, |s_i - s_j|, s_i + s_j] (192), symmetric.
// * z1 = phi W1 + b1, h1 = relu(z1) (128); z2 = h1 W2 + b2, h2 = relu(z2)
//   (128); out = h2 . w3 + b3, trained on log(1 + gain) with the loss
//   mean (out - y)^2 / 2 and Adam.
//
// Inference: BF16 MFMA (16x16x32) with FP32 accumulation, 16 pairs per
// wavefront; h1 goes through LDS (bf16) to become the second layer's A
// operand.  Training: FP32 tiled GEMMs and elementwise kernels, FP32 master
// weights; all reductions in a fixed order.
#include <math.h>

#include "common.hpp"
#include "ctx.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int SD = REC_SUR_SDIM;   // 64
constexpr int ND = 28;             // projections per half
constexpr int PH = 192, U1 = 128, U2 = 128;
constexpr int64_t OFF_W1 = 0, OFF_B1 = PH * U1, OFF_W2 = OFF_B1 + U1, OFF_B2 = OFF_W2 + U1 * U2,
                  OFF_W3 = OFF_B2 + U2, OFF_B3 = OFF_W3 + U2;
static_assert(OFF_B3 + 1 == REC_SUR_NPARAM, "parameter layout");

// ------------------------------------------------------------ sketches --
__global__ void k_proj_bits(uint64_t seed, int64_t Mp, uint32_t* bits) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Mp) return;
  uint32_t w = 0;
  for (int d = 0; d < ND; ++d)
    if (rec_ctr(seed, REC_STREAM_PROJ, (uint64_t)d, (uint64_t)s) >> 63) w |= 1u << d;
  bits[s] = w;
}

template <class R, int MODEL>
__global__ __launch_bounds__(256) void k_sketch(Fields F, const uint32_t* __restrict__ pbits,
                                                const int64_t* __restrict__ row_off,
                                                const double* __restrict__ colw, float* __restrict__ S,
                                                __bf16* __restrict__ Sb) {
  constexpr int NT = 256, NW = NT / REC_WAVE, NV = 2 * ND + 5;
  __shared__ double red[NW][NV];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const int64_t M = F.M, row = i * F.Mp;
  const R* H = reinterpret_cast<const R*>(F.H);
  const R* T = reinterpret_cast<const R*>(F.T);
  for (int64_t s = tid; s < M; s += NT) {
    double x, y, t, r, ha;
    if constexpr (MODEL == REC_GAUSS) {
      x = F.xf[row + s];
      y = x;
      r = (double)H[row + s];
      t = r;
      ha = fabs(r);
    } else {
      x = F.xs[row + s];
      y = MODEL == REC_KINETIC ? (double)F.ys[row + s] : x;
      t = (double)T[row + s];
      r = y - t;
      ha = fabs((double)H[row + s]);
    }
    const uint32_t pb = pbits[s];
    const double a = x + r, b = x - r;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const bool neg = (pb >> d) & 1u;
      acc[d] += neg ? -a : a;
      acc[ND + d] += neg ? -b : b;
    }
    acc[2 * ND + 0] += y;
    acc[2 * ND + 1] += t;
    acc[2 * ND + 2] += t * t;
    acc[2 * ND + 3] += ha;
    acc[2 * ND + 4] += r * r;
  }
  // fixed-order reduction: lanes by butterfly, then waves in order
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double v = rec_wave_sum(acc[q]);
    if ((tid & (REC_WAVE - 1)) == 0) red[tid / REC_WAVE][q] = v;
  }
  __syncthreads();
  if (tid < SD) {
    float out;
    const double inv = 1.0 / (double)M;
    if (tid < 2 * ND + 5) {
      double v = 0.0;
      for (int w = 0; w < NW; ++w) v += red[w][tid];
      if (tid < 2 * ND) out = (float)(v / sqrt((double)M));
      else if (tid == 2 * ND + 2) {
        double mt = 0.0, mt2 = 0.0;
        for (int w = 0; w < NW; ++w) { mt += red[w][2 * ND + 1]; mt2 += red[w][2 * ND + 2]; }
        out = (float)(mt2 * inv - (mt * inv) * (mt * inv));
      } else {
        out = (float)(v * inv);
      }
    } else {
      const int64_t e0 = row_off ? row_off[i] : 0, e1 = row_off ? row_off[i + 1] : 0;
      if (tid == 61) out = (float)log1p((double)(e1 - e0));
      else if (tid == 62) {
        double l1 = 0.0;
        for (int64_t e = e0; e < e1; ++e) l1 += fabs(colw[e]);
        out = (float)l1;
      } else {
        out = (float)F.theta[i];
      }
    }
    S[i * SD + tid] = out;
    Sb[i * SD + tid] = (__bf16)out;
  }
}

// -------------------------------------------------------------- inference --
// phi chunk of 8 features starting at feature f0 (f0 % 8 == 0) for (si, sj)
__device__ __forceinline__ void feat8(const float* si, const float* sj, int f0, float* o) {
  const int kind = f0 / SD, q0 = f0 % SD;
  const float4 a0 = *reinterpret_cast<const float4*>(si + q0);
  const float4 a1 = *reinterpret_cast<const float4*>(si + q0 + 4);
  const float4 b0 = *reinterpret_cast<const float4*>(sj + q0);
  const float4 b1 = *reinterpret_cast<const float4*>(sj + q0 + 4);
  const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  const float b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
  for (int v = 0; v < 8; ++v)
    o[v] = kind == 0 ? a[v] * b[v] : kind == 1 ? fabsf(a[v] - b[v]) : a[v] + b[v];
}

constexpr uint32_t OWNER_BIT = 0x80000000u;

// 64 pairs per block (4 waves x 16).  Lane l supplies pair l % 16 of its wave
// and the 8-wide k chunk l / 16 of each 32-wide step; the C fragment of a
// 16x16 block holds rows 4 (l / 16) + r, column l % 16.
__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ S,
                                                   const __bf16* __restrict__ W1t,
                                                   const __bf16* __restrict__ W2t,
                                                   const float* __restrict__ par, int64_t P,
                                                   const int32_t* __restrict__ I,
                                                   const int32_t* __restrict__ J,
                                                   const int32_t* __restrict__ Jmap,
                                                   const uint32_t* __restrict__ slot,
                                                   float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) __bf16 hb[4][16][U1 + 8];
  const int lane = threadIdx.x & (REC_WAVE - 1), w = threadIdx.x / REC_WAVE;
  const int pr = lane & 15, grp = lane >> 4;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + w) * 16;
  if (p0 >= P) return;   // whole wave: no block-level barrier below
  const int64_t p = p0 + pr;
  const bool valid = p < P && (slot == nullptr || (slot[p] & OWNER_BIT));
  int i = 0, j = 0;
  if (valid) {
    i = I[p];
    j = J[p];
    if (Jmap) j = Jmap[j];
  }
  const float* si = S + (int64_t)i * SD;
  const float* sj = S + (int64_t)j * SD;
  floatx4 acc[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < PH / 32; ++ks) {
    const int f0 = 32 * ks + 8 * grp;
    float fv[8];
    feat8(si, sj, f0, fv);
    bf16x8 a;
#pragma unroll
    for (int v = 0; v < 8; ++v) a[v] = (__bf16)fv[v];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(W1t + (int64_t)(nb * 16 + pr) * PH + f0);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
    }
  }
  // h1 = relu(z1 + b1) -> LDS (bf16), row = pair, column = unit
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) {
    const int u = nb * 16 + pr;
    const float bu = par[OFF_B1 + u];
#pragma unroll
    for (int r = 0; r < 4; ++r) hb[w][4 * grp + r][u] = (__bf16)fmaxf(acc[nb][r] + bu, 0.f);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  floatx4 acc2[8];
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) acc2[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < U1 / 32; ++ks) {
    const int k0 = 32 * ks + 8 * grp;
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&hb[w][pr][k0]);
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(W2t + (int64_t)(nb * 16 + pr) * U1 + k0);
      acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc2[nb], 0, 0, 0);
    }
  }
  // out = relu(z2 + b2) . w3 + b3: partial sums over this lane's 8 units, then
  // over the 16 lanes of the group (xor 1, 2, 4, 8 stays inside the group)
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nb = 0; nb < 8; ++nb) {
    const int v = nb * 16 + pr;
    const float bv = par[OFF_B2 + v], wv = par[OFF_W3 + v];
#pragma unroll
    for (int r = 0; r < 4; ++r) part[r] = fmaf(fmaxf(acc2[nb][r] + bv, 0.f), wv, part[r]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) part[r] += __shfl_xor(part[r], o, REC_WAVE);
  if (pr == 0) {
    const float b3 = par[OFF_B3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t q = p0 + 4 * grp + r;
      if (q < P) {
        const bool ok = slot == nullptr || (slot[q] & OWNER_BIT);
        out[q] = ok ? part[r] + b3 : -__builtin_inff();
      }
    }
  }
}

// bf16 copies of W1 and W2, transposed to [unit][input] for the B operand
__global__ void k_mlp_pack(const float* __restrict__ par, __bf16* __restrict__ W1t,
                           __bf16* __restrict__ W2t) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < PH * U1) {
    int f = (int)(e / U1), u = (int)(e % U1);
    W1t[(int64_t)u * PH + f] = (__bf16)par[OFF_W1 + e];
  } else if (e < PH * U1 + U1 * U2) {
    int64_t q = e - PH * U1;
    int a = (int)(q / U2), v = (int)(q % U2);
    W2t[(int64_t)v * U1 + a] = (__bf16)par[OFF_W2 + q];
  }
}

// --------------------------------------------------------------- training --
__global__ void k_pair_feat(const float* __restrict__ S, int64_t B, const int32_t* __restrict__ I,
                            const int32_t* __restrict__ J, float* __restrict__ phi) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * PH) return;
  int64_t b = e / PH;
  int f = (int)(e % PH), kind = f / SD, q = f % SD;
  float a = S[(int64_t)I[b] * SD + q], c = S[(int64_t)J[b] * SD + q];
  phi[e] = kind == 0 ? a * c : kind == 1 ? fabsf(a - c) : a + c;
}

// C[M x N] = op(A) op(B) (+ bias per column); A is M x K row-major (lda), or
// K x M when TA; B is K x N (ldb), or N x K when TB.  64 x 64 tiles, 256
// threads with 4 x 4 outputs each; the k sums run in a fixed order.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int lda, const float* __restrict__ Bm, int ldb,
                                              const float* __restrict__ bias, float* __restrict__ C,
                                              int ldc) {
  constexpr int T = 64, KS = 16;
  __shared__ float As[KS][T + 4];
  __shared__ float Bs[KS][T + 4];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
  float c[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += KS) {
    for (int q = threadIdx.x; q < KS * T; q += 256) {
      int kk = q / T, mm = q % T;
      int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < M && gk < K) va = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = va;
      int gn = n0 + mm;
      float vb = 0.f;
      if (gn < N && gk < K) vb = TB ? Bm[(int64_t)gn * ldb + gk] : Bm[(int64_t)gk * ldb + gn];
      Bs[kk][mm] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) { a[r] = As[kk][ty * 4 + r]; b[r] = Bs[kk][tx * 4 + r]; }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[r][q] = fmaf(a[r], b[q], c[r][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int gm = m0 + ty * 4 + r, gn = n0 + tx * 4 + q;
      if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = c[r][q] + (bias ? bias[gn] : 0.f);
    }
}

__global__ void k_relu(const float* __restrict__ z, float* __restrict__ h, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) h[e] = fmaxf(z[e], 0.f);
}

// out[b] = h2[b] . w3 + b3; dout[b] = (out - y) / B; per-row loss terms
__global__ void k_head(const float* __restrict__ h2, const float* __restrict__ par, int64_t B,
                       const float* __restrict__ y, float* __restrict__ out, float* __restrict__ dout,
                       double* __restrict__ lterm) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float s = par[OFF_B3];
  for (int v = 0; v < U2; ++v) s = fmaf(h2[b * U2 + v], par[OFF_W3 + v], s);
  out[b] = s;
  if (y) {
    float d = s - y[b];
    dout[b] = d / (float)B;
    lterm[b] = 0.5 * (double)d * (double)d;
  }
}

// dz2 = dout (x) w3 * (z2 > 0)
__global__ void k_dz2(const float* __restrict__ dout, const float* __restrict__ par,
                      const float* __restrict__ z2, int64_t B, float* __restrict__ dz2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * U2) return;
  int v = (int)(e % U2);
  dz2[e] = z2[e] > 0.f ? dout[e / U2] * par[OFF_W3 + v] : 0.f;
}

__global__ void k_mask_relu(float* __restrict__ d, const float* __restrict__ z, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(z[e] > 0.f)) d[e] = 0.f;
}

// column sums of a B x n matrix (optionally weighted by wt[b]), fixed order
__global__ void k_colsum(const float* __restrict__ a, const float* __restrict__ wt, int64_t B, int n,
                         float* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float s = 0.f;
  for (int64_t b = 0; b < B; ++b) s = fmaf(a[b * n + c], wt ? wt[b] : 1.f, s);
  out[c] = s;
}

__global__ void k_sum_f(const float* __restrict__ a, int64_t n, float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (int64_t b = 0; b < n; ++b) s += a[b];
  *out = s;
}

__global__ void k_sum_d(const double* __restrict__ a, int64_t n, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += blockDim.x) s += a[b];
  s = rec_wave_sum(s);
  if ((threadIdx.x & (REC_WAVE - 1)) == 0) sh[threadIdx.x / REC_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / REC_WAVE); ++w) t += sh[w];
    *out = t / (double)n;
  }
}

// Adam (Kingma & Ba 2015) with bias correction; c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float gm = b1 * m[e] + (1.f - b1) * g[e];
  float gv = b2 * v[e] + (1.f - b2) * g[e] * g[e];
  m[e] = gm;
  v[e] = gv;
  p[e] -= lr * (gm / c1) / (sqrtf(gv / c2) + eps);
}

// He-uniform initial weights from the counter generator (stream 8), zero biases
__global__ void k_mlp_init(float* __restrict__ p, uint64_t seed) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= REC_SUR_NPARAM) return;
  float fan = 0.f;
  if (e < OFF_B1) fan = PH;
  else if (e >= OFF_W2 && e < OFF_B2) fan = U1;
  else if (e >= OFF_W3 && e < OFF_B3) fan = U2;
  if (fan == 0.f) { p[e] = 0.f; return; }
  uint64_t r = rec_ctr(seed, REC_STREAM_INIT_W, (uint64_t)e, 0);
  float u = (float)((double)(r >> 11) * 0x1.0p-53) * 2.f - 1.f;
  p[e] = u * sqrtf(6.f / fan);
}

inline int64_t gr(int64_t n, int b = 256) { return (n + b - 1) / b; }

template <bool TA, bool TB>
void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
          const float* bias, float* C, int ldc) {
  dim3 g((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm<TA, TB>), g, dim3(256), 0, s, M, N, K, A, lda, B, ldb, bias, C, ldc);
}

}  // namespace

rec_status rec_sur_init(rec_ctx* ctx) {
  hipStream_t s = ctx->stream;
  hipLaunchKernelGGL(k_proj_bits, dim3(gr(ctx->F.Mp)), dim3(256), 0, s, ctx->cfg.seed, ctx->F.Mp,
                     ctx->sur_pbits);
  hipLaunchKernelGGL(k_mlp_init, dim3(gr(REC_SUR_NPARAM)), dim3(256), 0, s, ctx->sur_par, ctx->cfg.seed);
  REC_HIP(hipMemsetAsync(ctx->sur_m, 0, REC_SUR_NPARAM * sizeof(float), s));
  REC_HIP(hipMemsetAsync(ctx->sur_v, 0, REC_SUR_NPARAM * sizeof(float), s));
  ctx->sur_t = 0;
  return rec_sur_pack(ctx);
}

rec_status rec_sur_pack(rec_ctx* ctx) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(gr(PH * U1 + U1 * U2)), dim3(256), 0, ctx->stream, ctx->sur_par,
                     ctx->sur_w1t, ctx->sur_w2t);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_sur_sketch(rec_ctx* ctx) {
  hipStream_t s = ctx->stream;
  const int64_t N = ctx->cfg.N;
#define REC_SK(R, MOD)                                                                           \
  hipLaunchKernelGGL((k_sketch<R, MOD>), dim3(N), dim3(256), 0, s, ctx->F, ctx->sur_pbits,       \
                     ctx->row_off, ctx->colw, ctx->sur_S, ctx->sur_Sb)
  if (ctx->fp32) {
    if (ctx->cfg.model == REC_ISING) REC_SK(float, REC_ISING);
    else if (ctx->cfg.model == REC_GAUSS) REC_SK(float, REC_GAUSS);
    else REC_SK(float, REC_KINETIC);
  } else {
    if (ctx->cfg.model == REC_ISING) REC_SK(double, REC_ISING);
    else if (ctx->cfg.model == REC_GAUSS) REC_SK(double, REC_GAUSS);
    else REC_SK(double, REC_KINETIC);
  }
#undef REC_SK
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_sur_infer(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                         const int32_t* Jmap, const uint32_t* slot, float* out) {
  if (P <= 0) return REC_OK;
  const int64_t blocks = (P + 63) / 64;
  hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(256), 0, ctx->stream, ctx->sur_S, ctx->sur_w1t,
                     ctx->sur_w2t, ctx->sur_par, P, I, J, Jmap, slot, out);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

// Forward and backward of the batch (FP32); gradient into ctx->sur_g, mean
// loss into ctx->dresult[8].
rec_status rec_sur_grad(rec_ctx* ctx, int64_t B, const int32_t* I, const int32_t* J, const float* y) {
  hipStream_t s = ctx->stream;
  if (B <= 0 || B > REC_SUR_BATCH) { ctx->err = "batch size out of range"; return REC_E_INVAL; }
  float* par = ctx->sur_par;
  float* g = ctx->sur_g;
  float* phi = ctx->sur_phi;
  float *z1 = ctx->sur_z1, *h1 = ctx->sur_h1, *z2 = ctx->sur_z2, *h2 = ctx->sur_h2;
  float *out = ctx->sur_out, *dout = ctx->sur_dout;
  const int Bi = (int)B;
  hipLaunchKernelGGL(k_pair_feat, dim3(gr(B * PH)), dim3(256), 0, s, ctx->sur_S, B, I, J, phi);
  gemm<false, false>(s, Bi, U1, PH, phi, PH, par + OFF_W1, U1, par + OFF_B1, z1, U1);
  hipLaunchKernelGGL(k_relu, dim3(gr(B * U1)), dim3(256), 0, s, z1, h1, B * U1);
  gemm<false, false>(s, Bi, U2, U1, h1, U1, par + OFF_W2, U2, par + OFF_B2, z2, U2);
  hipLaunchKernelGGL(k_relu, dim3(gr(B * U2)), dim3(256), 0, s, z2, h2, B * U2);
  hipLaunchKernelGGL(k_head, dim3(gr(B)), dim3(256), 0, s, h2, par, B, y, out, dout, ctx->sur_lterm);
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(256), 0, s, ctx->sur_lterm, B, ctx->dresult + 8);
  // head gradients
  hipLaunchKernelGGL(k_colsum, dim3(gr(U2)), dim3(256), 0, s, h2, dout, B, U2, g + OFF_W3);
  hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(64), 0, s, dout, B, g + OFF_B3);
  // layer 2 (h2 is dead after the head gradient: it holds dz2 from here)
  hipLaunchKernelGGL(k_dz2, dim3(gr(B * U2)), dim3(256), 0, s, dout, par, z2, B, h2);
  gemm<true, false>(s, U1, U2, Bi, h1, U1, h2, U2, nullptr, g + OFF_W2, U2);
  hipLaunchKernelGGL(k_colsum, dim3(gr(U2)), dim3(256), 0, s, h2, nullptr, B, U2, g + OFF_B2);
  // layer 1: dz1 = (dz2 W2^T) * (z1 > 0)
  gemm<false, true>(s, Bi, U1, U2, h2, U2, par + OFF_W2, U2, nullptr, h1, U1);   // h1 := dh1
  hipLaunchKernelGGL(k_mask_relu, dim3(gr(B * U1)), dim3(256), 0, s, h1, z1, B * U1);
  gemm<true, false>(s, PH, U1, Bi, phi, PH, h1, U1, nullptr, g + OFF_W1, U1);
  hipLaunchKernelGGL(k_colsum, dim3(gr(U1)), dim3(256), 0, s, h1, nullptr, B, U1, g + OFF_B1);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_sur_adam(rec_ctx* ctx, float lr) {
  ctx->sur_t += 1;
  const double c1 = 1.0 - std::pow(0.9, (double)ctx->sur_t);
  const double c2 = 1.0 - std::pow(0.999, (double)ctx->sur_t);
  hipLaunchKernelGGL(k_adam, dim3(gr(REC_SUR_NPARAM)), dim3(256), 0, ctx->stream, ctx->sur_par, ctx->sur_g,
                     ctx->sur_m, ctx->sur_v, (int64_t)REC_SUR_NPARAM, lr, (float)c1, (float)c2);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

// ------------------------------------------------------- search filter --
// Candidates of one NNDescent chunk: (gi[p], S[v[p]]) with slot words whose
// top bit marks the pairs this chunk scores.  flag[p]: 0 not scored here,
// 1 kept, 2 below the threshold but scored (audit sample, or every one in
// shadow mode), 3 dropped (its cache value becomes NaN: never scored in this
// FindBest call, ranked last by every list).
namespace {

__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u >> 31) ? ~u : (u | 0x80000000u);
}

constexpr int SUR_BINS = 4096;

__global__ __launch_bounds__(256) void k_sur_hist(const float* __restrict__ pred,
                                                  const uint32_t* __restrict__ slot, int64_t n,
                                                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t hs[SUR_BINS];
  for (int q = threadIdx.x; q < SUR_BINS; q += 256) hs[q] = 0;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
    if (slot[p] & OWNER_BIT) atomicAdd(&hs[ord_f32(pred[p]) >> 20], 1u);
  __syncthreads();
  for (int q = threadIdx.x; q < SUR_BINS; q += 256)
    if (hs[q]) atomicAdd(&hist[q], hs[q]);
}

// thr = lower edge (ordered key) of the bin where the count from the top
// reaches ceil(rho * owned)
__global__ void k_sur_thr(const uint32_t* hist, double rho, uint32_t* thr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t tot = 0;
  for (int q = 0; q < SUR_BINS; ++q) tot += hist[q];
  const uint64_t want = (uint64_t)ceil(rho * (double)tot);
  uint64_t cum = 0;
  uint32_t t = 0;
  for (int q = SUR_BINS - 1; q >= 0; --q) {
    cum += hist[q];
    if (cum >= want) { t = (uint32_t)q << 20; break; }
  }
  *thr = t;
}

__global__ void k_sur_filter(const float* __restrict__ pred, uint32_t* __restrict__ slot,
                             const int32_t* __restrict__ gi, const int32_t* __restrict__ v,
                             const int32_t* __restrict__ S, int64_t n, const uint32_t* __restrict__ thr,
                             Cache C, int shadow, uint64_t seed, uint32_t audit_mask,
                             uint8_t* __restrict__ flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t sw = slot[p];
  if (!(sw & OWNER_BIT)) { flag[p] = 0; return; }
  if (ord_f32(pred[p]) >= *thr) { flag[p] = 1; return; }
  if (shadow) { flag[p] = 2; return; }
  const uint64_t key = rec_pair_key(gi[p], S[v[p]], false);
  if ((rec_ctr(seed, REC_STREAM_AUDIT, key, 1) & audit_mask) == 0) { flag[p] = 2; return; }
  flag[p] = 3;
  const uint32_t s = sw & ~OWNER_BIT;
  const uint64_t cap = C.mask + 1;
  if (s < cap) C.vals[s] = __builtin_nan("");
  else C.ovf[s - cap] = __builtin_nan("");
  slot[p] = s;   // not scored by this chunk
}

// after scoring: positives among kept (cnt[0]) and among scored-below-threshold (cnt[1])
__global__ void k_sur_count(const uint32_t* __restrict__ slot, const uint8_t* __restrict__ flag,
                            int64_t n, Cache C, int64_t* cnt) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int kp = 0, dp = 0, kt = 0, dt = 0, dr = 0;
  if (p < n) {
    const uint8_t f = flag[p];
    if (f == 1 || f == 2) {
      const uint32_t s = slot[p] & ~OWNER_BIT;
      const uint64_t cap = C.mask + 1;
      const double g = s < cap ? C.vals[s] : C.ovf[s - cap];
      const bool pos = g > 0.0;
      kp = f == 1 && pos;
      dp = f == 2 && pos;
      kt = f == 1;
      dt = f == 2;
    }
    dr = f == 3;
  }
  kp = rec_wave_sum(kp); dp = rec_wave_sum(dp); kt = rec_wave_sum(kt); dt = rec_wave_sum(dt);
  dr = rec_wave_sum(dr);
  if (rec_lane() == 0) {
    if (kp) atomicAdd((unsigned long long*)&cnt[0], (unsigned long long)kp);
    if (dp) atomicAdd((unsigned long long*)&cnt[1], (unsigned long long)dp);
    if (kt) atomicAdd((unsigned long long*)&cnt[2], (unsigned long long)kt);
    if (dt) atomicAdd((unsigned long long*)&cnt[3], (unsigned long long)dt);
    if (dr) atomicAdd((unsigned long long*)&cnt[4], (unsigned long long)dr);
  }
}

// training records from the score cache: every positive gain (up to cap_pos,
// at [0, cap_pos)) and the zero gains whose pair hash falls in a 1/2^zbits
// sample (up to cap_zero, at [zoff, zoff + cap_zero))
__global__ void k_sur_collect(Cache C, uint64_t seed, int zbits, int32_t* __restrict__ ri,
                              int32_t* __restrict__ rj, float* __restrict__ ry, int64_t* cur,
                              int64_t cap_pos, int64_t cap_zero, int64_t zoff) {
  uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t cap = C.mask + 1;
  uint64_t key = s < cap ? C.keys[s] : REC_EMPTY;
  if (key != REC_EMPTY) key &= ~0xFF000000FF000000ULL;   // drop the search-level tags
  double g = key != REC_EMPTY ? C.vals[s] : 0.0;
  const bool ok = key != REC_EMPTY && g == g;
  const bool pos = ok && g > 0.0;
  const bool zero = ok && !(g > 0.0) &&
                    (rec_ctr(seed, REC_STREAM_AUDIT, key, 2) & ((1ull << zbits) - 1)) == 0;
  int64_t a = rec_append(&cur[0], pos);
  if (a >= 0 && a < cap_pos) {
    ri[a] = (int32_t)(key >> 32);
    rj[a] = (int32_t)(key & 0xffffffffu);
    ry[a] = (float)log1p(g);
  }
  int64_t b = rec_append(&cur[1], zero);
  if (b >= 0 && b < cap_zero) {
    ri[zoff + b] = (int32_t)(key >> 32);
    rj[zoff + b] = (int32_t)(key & 0xffffffffu);
    ry[zoff + b] = 0.f;
  }
}

}  // namespace

rec_status rec_sur_filter(rec_ctx* ctx, int64_t n, const int32_t* gi, const int32_t* v,
                          const int32_t* S, uint32_t* slot, int shadow) {
  if (n <= 0) return REC_OK;
  hipStream_t s = ctx->stream;
  rec_status st = rec_sur_infer(ctx, n, gi, v, S, slot, ctx->sur_pred);
  if (st != REC_OK) return st;
  REC_HIP(hipMemsetAsync(ctx->sur_hist, 0, SUR_BINS * sizeof(uint32_t), s));
  const int64_t hb = std::min<int64_t>(gr(n), 2048);
  hipLaunchKernelGGL(k_sur_hist, dim3(hb), dim3(256), 0, s, ctx->sur_pred, slot, n, ctx->sur_hist);
  hipLaunchKernelGGL(k_sur_thr, dim3(1), dim3(64), 0, s, ctx->sur_hist, ctx->sur_rho, ctx->sur_thr);
  hipLaunchKernelGGL(k_sur_filter, dim3(gr(n)), dim3(256), 0, s, ctx->sur_pred, slot, gi, v, S, n,
                     ctx->sur_thr, ctx->C, shadow, ctx->cfg.seed, (uint32_t)(ctx->sur_audit - 1),
                     ctx->sur_flag);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_sur_count(rec_ctx* ctx, int64_t n, const uint32_t* slot) {
  if (n <= 0) return REC_OK;
  hipLaunchKernelGGL(k_sur_count, dim3(gr(n)), dim3(256), 0, ctx->stream, slot, ctx->sur_flag, n,
                     ctx->C, ctx->sur_cnt);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

// Records from the cache of the FindBest call that just ended, then Adam
// steps on them (full batch: positives first, then the zero sample).
rec_status rec_sur_collect_train(rec_ctx* ctx, double* loss, int64_t* npos, int64_t* nzero) {
  hipStream_t s = ctx->stream;
  const int64_t cp = REC_SUR_BATCH / 4, cz = REC_SUR_BATCH - REC_SUR_BATCH / 4;
  int64_t* cur = ctx->sur_cnt + 8;
  REC_HIP(hipMemsetAsync(cur, 0, 2 * sizeof(int64_t), s));
  const uint64_t cap = ctx->C.mask + 1;
  // record arrays hold 2 * REC_SUR_BATCH: positives at [0, cp), zeros at
  // [REC_SUR_BATCH, REC_SUR_BATCH + cz); the zeros are then moved down behind
  // the positives (disjoint ranges: np + nz <= REC_SUR_BATCH)
  const int64_t zoff = REC_SUR_BATCH;
  hipLaunchKernelGGL(k_sur_collect, dim3((cap + 255) / 256), dim3(256), 0, s, ctx->C, ctx->cfg.seed,
                     ctx->sur_zbits, ctx->sur_ri, ctx->sur_rj, ctx->sur_ry, cur, cp, cz, zoff);
  int64_t h[2];
  REC_HIP(hipMemcpyAsync(h, cur, sizeof(h), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  const int64_t np = std::min(h[0], cp), nz = std::min(h[1], cz);
  *npos = np;
  *nzero = nz;
  if (np + nz == 0) { *loss = 0.0; return REC_OK; }
  // pack positives then zeros contiguously
  if (nz > 0) {
    REC_HIP(hipMemcpyAsync(ctx->sur_ri + np, ctx->sur_ri + zoff, nz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    REC_HIP(hipMemcpyAsync(ctx->sur_rj + np, ctx->sur_rj + zoff, nz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    REC_HIP(hipMemcpyAsync(ctx->sur_ry + np, ctx->sur_ry + zoff, nz * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  const int64_t B = np + nz;
  for (int st = 0; st < ctx->sur_steps; ++st) {
    rec_status r = rec_sur_grad(ctx, B, ctx->sur_ri, ctx->sur_rj, ctx->sur_ry);
    if (r != REC_OK) return r;
    if ((r = rec_sur_adam(ctx, ctx->sur_lr)) != REC_OK) return r;
  }
  rec_status r = rec_sur_pack(ctx);
  if (r != REC_OK) return r;
  REC_HIP(hipMemcpyAsync(loss, ctx->dresult + 8, sizeof(double), hipMemcpyDeviceToHost, s));
  REC_HIP(hipStreamSynchronize(s));
  return REC_OK;
}
