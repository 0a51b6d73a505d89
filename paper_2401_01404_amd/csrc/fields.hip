// Data layout, fields, theta and the objective.
//
// Layout: node-major rows padded to Mp = 64 * npl samples (zeros past M), so
// a wavefront reads whole rows with one contiguous block per load.
//
// Fields [App. A, "keeping track of the weighted sum of the neighbors"]:
// m_i = sum_{j != i} W_ij x_j per sample, summed in FP64 over the sorted
// row list of W and rounded once to the working precision; Ising and kinetic
// store h = theta + m, t = tanh h and the int8 copy of y - t, the Gaussian model stores the residual
// r = x + theta^2 m.
//
// Objective [App. A]: sum over nodes and samples of the log conditional plus
// the L1 prior -lambda sum |W_ij|, summed in FP64 in a fixed order (per-row
// partials, then one block), so repeated evaluations give the same bits.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "ctx.hpp"

namespace {

constexpr int FT = 256;   // threads per row block

template <class R> __device__ __forceinline__ R tanh_(R x);
template <> __device__ __forceinline__ float tanh_<float>(float x) { return tanhf(x); }
template <> __device__ __forceinline__ double tanh_<double>(double x) { return tanh(x); }

// log(2 cosh h) in the working precision, stable for large |h|
__device__ __forceinline__ float log2cosh_(float h) {
  float a = fabsf(h);
  return a + log1pf(__expf(-2.f * a));
}
__device__ __forceinline__ double log2cosh_(double h) {
  double a = fabs(h);
  return a + log1p(exp(-2.0 * a));
}

__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  v = rec_wave_sum(v);
  if ((tid & (REC_WAVE - 1)) == 0) sh[tid / REC_WAVE] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    for (int w = 0; w < FT / REC_WAVE; ++w) s += sh[w];
    sh[0] = s;
  }
  __syncthreads();
  s = sh[0];
  __syncthreads();
  return s;
}

// X (caller layout) -> padded int8 rows; kinetic: input side columns 0..M-1,
// target side columns 1..M.  Flags any value other than +-1.
__global__ __launch_bounds__(FT) void k_load_int8(const int8_t* __restrict__ X, int64_t ldx,
                                                  int64_t M, int64_t Mp, int kinetic,
                                                  int8_t* __restrict__ xs, int8_t* __restrict__ ys,
                                                  int32_t* err) {
  const int64_t i = blockIdx.x;
  for (int64_t s = threadIdx.x; s < Mp; s += FT) {
    int8_t a = 0, b = 0;
    if (s < M) {
      a = X[i * ldx + s];
      b = kinetic ? X[i * ldx + s + 1] : a;
      if ((a != 1 && a != -1) || (b != 1 && b != -1)) atomicOr(err, 4);
    }
    xs[i * Mp + s] = a;
    if (kinetic) ys[i * Mp + s] = b;
  }
}

// Lane words of the screen: bit c*VEC + k of lane l = sample
// c*64*VEC + l*VEC + k is +1 (one wave per node).
__global__ __launch_bounds__(REC_WAVE) void k_pack_bits(const int8_t* __restrict__ x, int64_t Mp,
                                                        int npl, void* __restrict__ q) {
  const int64_t i = blockIdx.x;
  const int l = threadIdx.x;
  const int vec = npl < 4 ? npl : 4, ch = npl / vec;
  uint32_t w = 0;
  for (int c = 0; c < ch; ++c)
    for (int k = 0; k < vec; ++k) {
      int64_t s = (int64_t)c * REC_WAVE * vec + (int64_t)l * vec + k;
      if (x[i * Mp + s] > 0) w |= 1u << (c * vec + k);
    }
  if (npl <= 16)
    reinterpret_cast<uint16_t*>(q)[i * REC_WAVE + l] = (uint16_t)w;
  else
    reinterpret_cast<uint32_t*>(q)[i * REC_WAVE + l] = w;
}

__global__ __launch_bounds__(FT) void k_load_f32(const float* __restrict__ X, int64_t ldx, int64_t M,
                                                 int64_t Mp, float* __restrict__ xf,
                                                 double* __restrict__ sq, int32_t* err) {
  __shared__ double sh[FT / REC_WAVE];
  const int64_t i = blockIdx.x;
  double s2 = 0.0;
  for (int64_t s = threadIdx.x; s < Mp; s += FT) {
    float a = 0.f;
    if (s < M) {
      a = X[i * ldx + s];
      if (!isfinite(a)) atomicOr(err, 4);
      s2 += (double)a * (double)a;
    }
    xf[i * Mp + s] = a;
  }
  double tot = block_sum(s2, sh);
  if (threadIdx.x == 0) sq[i] = tot;
}

// One wavefront per row; lane l holds the samples c * 64 * VEC + l * VEC + k
// (k < VEC, c < NPL / VEC), so each load or store of the wave covers one
// contiguous run of the row.
template <int NPL> struct RowLayout {
  static constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  __device__ static int64_t at(int c, int lane) { return (int64_t)c * (REC_WAVE * VEC) + (int64_t)lane * VEC; }
};

template <class T, int VEC> struct alignas(sizeof(T) * VEC) Pack { T v[VEC]; };

template <int VEC>
__device__ __forceinline__ void ld_i8(const int8_t* p, double* o) {
  const Pack<int8_t, VEC> q = *reinterpret_cast<const Pack<int8_t, VEC>*>(p);
#pragma unroll
  for (int k = 0; k < VEC; ++k) o[k] = (double)q.v[k];
}
template <int VEC>
__device__ __forceinline__ void ld_f32(const float* p, double* o) {
  const Pack<float, VEC> q = *reinterpret_cast<const Pack<float, VEC>*>(p);
#pragma unroll
  for (int k = 0; k < VEC; ++k) o[k] = (double)q.v[k];
}

// Rebuild the fields of row i from its sorted W row list (summed over the
// list in order, per sample, in FP64; rounded once).  Padding samples get
// h = t = 0 (their x and y are 0).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(FT) void k_fields(Fields F, const int64_t* __restrict__ row_off,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ colw) {
  using L = RowLayout<NPL>;
  constexpr int VEC = L::VEC, CH = L::CH;
  const int lane = threadIdx.x & (REC_WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * (FT / REC_WAVE) + threadIdx.x / REC_WAVE;
  if (i >= F.N) return;
  const int64_t e0 = row_off ? row_off[i] : 0, e1 = row_off ? row_off[i + 1] : 0;
  double acc[NPL];
#pragma unroll
  for (int q = 0; q < NPL; ++q) acc[q] = 0.0;
  for (int64_t e = e0; e < e1; ++e) {
    const int64_t j = col[e];
    const double w = colw[e];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      double x[VEC];
      if (MODEL == REC_GAUSS) ld_f32<VEC>(F.xf + j * F.Mp + L::at(c, lane), x);
      else ld_i8<VEC>(F.xs + j * F.Mp + L::at(c, lane), x);
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[c * VEC + k] += w * x[k];
    }
  }
  const double th = F.theta[i];
  R* H = reinterpret_cast<R*>(F.H);
  R* T = reinterpret_cast<R*>(F.T);
  constexpr int UW = rec_u4_words(NPL);
  uint32_t uw[UW];
#pragma unroll
  for (int w = 0; w < UW; ++w) uw[w] = 0u;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = L::at(c, lane), idx = i * F.Mp + o;
    Pack<R, VEC> hv, tv;
    Pack<int8_t, VEC> rv;
    if (MODEL == REC_GAUSS) {
      double x[VEC];
      ld_f32<VEC>(F.xf + idx, x);
#pragma unroll
      for (int k = 0; k < VEC; ++k) hv.v[k] = o + k < F.M ? (R)(x[k] + th * th * acc[c * VEC + k]) : R(0);
      *reinterpret_cast<Pack<R, VEC>*>(H + idx) = hv;
    } else {
      const int8_t* Y = MODEL == REC_KINETIC ? F.ys : F.xs;
      double y[VEC];
      ld_i8<VEC>(Y + idx, y);
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const bool in = o + k < F.M;
        const R h = in ? (R)(th + acc[c * VEC + k]) : R(0);
        const R t = in ? tanh_<R>(h) : R(0);
        hv.v[k] = h;
        tv.v[k] = t;
        rv.v[k] = rec_q8((float)((R)y[k] - t));
        const int n = c * VEC + k;
        if (in) uw[n >> 3] |= rec_u4((float)(R(1) - (R)y[k] * t)) << (4 * (n & 7));
      }
      *reinterpret_cast<Pack<R, VEC>*>(H + idx) = hv;
      *reinterpret_cast<Pack<R, VEC>*>(T + idx) = tv;
      *reinterpret_cast<Pack<int8_t, VEC>*>(F.rq + idx) = rv;
    }
  }
  if (MODEL != REC_GAUSS) {
#pragma unroll
    for (int w = 0; w < UW; ++w) F.u4[(i * UW + w) * REC_WAVE + lane] = uw[w];
  }
}

// Refit theta_i [App. A, theta updated alongside W], one wavefront per row
// with the row's samples held in registers:
//   Ising / kinetic: root of sum_m (y_m - tanh(theta + m_m)) on [-8, 8]
//   (Newton inside the bracket, bisection otherwise), m = h - theta_old;
//   Gaussian: v = theta^2 is the positive root of C v^2 + M v - A = 0,
//   A = sum x^2, C = sum m^2, m = (r - x) / theta_old^2.
// Then the row's fields are shifted to the new theta.
//
// With row_off given, the row's coupling sums m are first formed from its
// sorted W row list in registers (FP64, in the order k_fields sums them); the
// refit uses them unrounded, and the fields written at the new theta are the
// ones k_fields computes there, bit for bit.  The fields are then written
// once instead of twice, and a later rebuild from (W, theta) reproduces them.
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(FT) void k_theta(Fields F, const int64_t* __restrict__ row_off,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ colw) {
  using L = RowLayout<NPL>;
  constexpr int VEC = L::VEC, CH = L::CH;
  const int lane = threadIdx.x & (REC_WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * (FT / REC_WAVE) + threadIdx.x / REC_WAVE;
  if (i >= F.N) return;
  const double th0 = F.theta[i];
  R* H = reinterpret_cast<R*>(F.H);
  R* T = reinterpret_cast<R*>(F.T);
  const int8_t* Y = MODEL == REC_KINETIC ? F.ys : F.xs;
  double mm[NPL], y[NPL];
  double acc[NPL];
#pragma unroll
  for (int q = 0; q < NPL; ++q) acc[q] = 0.0;
  if (row_off) {
    for (int64_t e = row_off[i]; e < row_off[i + 1]; ++e) {
      const int64_t j = col[e];
      const double w = colw[e];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        double x[VEC];
        if (MODEL == REC_GAUSS) ld_f32<VEC>(F.xf + j * F.Mp + L::at(c, lane), x);
        else ld_i8<VEC>(F.xs + j * F.Mp + L::at(c, lane), x);
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc[c * VEC + k] += w * x[k];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = L::at(c, lane), idx = i * F.Mp + o;
    if (MODEL == REC_GAUSS) ld_f32<VEC>(F.xf + idx, y + c * VEC);
    else ld_i8<VEC>(Y + idx, y + c * VEC);
    Pack<R, VEC> hv;
    if (row_off) {
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        hv.v[k] = o + k < F.M ? (MODEL == REC_GAUSS ? (R)(y[c * VEC + k] + th0 * th0 * acc[c * VEC + k])
                                                    : (R)(th0 + acc[c * VEC + k]))
                              : R(0);
    } else {
      hv = *reinterpret_cast<const Pack<R, VEC>*>(H + idx);
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const double hh = (double)hv.v[k];
      // rebuilt rows keep the unrounded coupling sums, so the fields written
      // below are the ones k_fields computes at the new theta, bit for bit
      mm[c * VEC + k] = row_off ? acc[c * VEC + k]
                                : (MODEL == REC_GAUSS ? (hh - y[c * VEC + k]) / (th0 * th0) : hh - th0);
    }
  }
  auto valid = [&](int q) { return L::at(q / VEC, lane) + q % VEC < F.M; };
  double th = th0;
  if (MODEL == REC_GAUSS) {
    double A = 0.0, C = 0.0;
#pragma unroll
    for (int q = 0; q < NPL; ++q)
      if (valid(q)) {
        A += y[q] * y[q];
        C += mm[q] * mm[q];
      }
    A = rec_wave_sum(A);
    C = rec_wave_sum(C);
    const double M = (double)F.M;
    const double v = C > 0 ? (-M + sqrt(M * M + 4.0 * A * C)) / (2.0 * C) : A / M;
    th = sqrt(v);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t idx = i * F.Mp + L::at(c, lane);
      Pack<R, VEC> hv;
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        hv.v[k] = valid(c * VEC + k) ? (R)(y[c * VEC + k] + th * th * mm[c * VEC + k]) : R(0);
      *reinterpret_cast<Pack<R, VEC>*>(H + idx) = hv;
    }
  } else {
    auto eval = [&](double t, double& f, double& df) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int q = 0; q < NPL; ++q)
        if (valid(q)) {
          const R tt = tanh_<R>((R)(t + mm[q]));
          a += y[q] - (double)tt;
          b -= 1.0 - (double)tt * (double)tt;
        }
      f = rec_wave_sum(a);
      df = rec_wave_sum(b);
    };
    const double TMAX = 8.0;
    double f, df;
    eval(TMAX, f, df);
    if (f >= 0) th = TMAX;
    else {
      eval(-TMAX, f, df);
      if (f <= 0) th = -TMAX;
      else {
        double lo = -TMAX, hi = TMAX;
        double t = fmin(fmax(th0, lo), hi);
        eval(t, f, df);
        for (int it = 0; it < 100; ++it) {
          if (f == 0.0) break;
          if (f > 0) lo = t; else hi = t;
          double tn = df < 0 ? t - f / df : 0.5 * (lo + hi);
          if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
          const double step = tn - t;
          t = tn;
          if (fabs(step) <= (sizeof(R) == 4 ? 1e-9 : 1e-15) * fmax(1.0, fabs(t)) || hi - lo < 1e-300)
            break;
          eval(t, f, df);
        }
        th = t;
      }
    }
    constexpr int UW = rec_u4_words(NPL);
    uint32_t uw[UW];
#pragma unroll
    for (int w = 0; w < UW; ++w) uw[w] = 0u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t idx = i * F.Mp + L::at(c, lane);
      Pack<R, VEC> hv, tv;
      Pack<int8_t, VEC> rv;
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const bool in = valid(c * VEC + k);
        const R h = in ? (R)(th + mm[c * VEC + k]) : R(0);
        const R t = in ? tanh_<R>(h) : R(0);
        hv.v[k] = h;
        tv.v[k] = t;
        rv.v[k] = rec_q8((float)((R)y[c * VEC + k] - t));
        const int n = c * VEC + k;
        if (in) uw[n >> 3] |= rec_u4((float)(R(1) - (R)y[c * VEC + k] * t)) << (4 * (n & 7));
      }
      *reinterpret_cast<Pack<R, VEC>*>(H + idx) = hv;
      *reinterpret_cast<Pack<R, VEC>*>(T + idx) = tv;
      *reinterpret_cast<Pack<int8_t, VEC>*>(F.rq + idx) = rv;
    }
#pragma unroll
    for (int w = 0; w < UW; ++w) F.u4[(i * UW + w) * REC_WAVE + lane] = uw[w];
  }
  if (lane == 0) F.theta[i] = th;
}

// Per-row log pseudolikelihood into part[i] (one wavefront per row).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(FT) void k_rowll(Fields F, double* part) {
  using L = RowLayout<NPL>;
  constexpr int VEC = L::VEC, CH = L::CH;
  const int lane = threadIdx.x & (REC_WAVE - 1);
  const int64_t i = (int64_t)blockIdx.x * (FT / REC_WAVE) + threadIdx.x / REC_WAVE;
  if (i >= F.N) return;
  const R* H = reinterpret_cast<const R*>(F.H);
  const int8_t* Y = MODEL == REC_KINETIC ? F.ys : F.xs;
  const double v = MODEL == REC_GAUSS ? F.theta[i] * F.theta[i] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = L::at(c, lane), idx = i * F.Mp + o;
    const Pack<R, VEC> hv = *reinterpret_cast<const Pack<R, VEC>*>(H + idx);
    double y[VEC];
    if (MODEL != REC_GAUSS) ld_i8<VEC>(Y + idx, y);
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      if (o + k >= F.M) continue;
      const R h = hv.v[k];
      if (MODEL == REC_GAUSS) acc += -(double)h * (double)h / (2.0 * v);
      else acc += (double)((R)y[k] * h - log2cosh_(h));
    }
  }
  acc = rec_wave_sum(acc);
  if (lane == 0) {
    if (MODEL == REC_GAUSS) acc += (double)F.M * (-log(F.theta[i]) - 0.5 * log(2.0 * M_PI));
    part[i] = acc;
  }
}

// Sum part[0..n) in a fixed order (one block, strided loads): *out = the sum
__global__ __launch_bounds__(FT) void k_sum(const double* part, int64_t n, double* out) {
  __shared__ double sh[FT / REC_WAVE];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += FT) acc += part[k];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

// sum |w| over the sorted W list, strided like k_sum_partial
__global__ __launch_bounds__(FT) void k_abs_partial(const double* w, int64_t n, double* part,
                                                    int64_t nchunk) {
  int64_t c = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (c >= nchunk) return;
  double acc = 0.0;
  for (int64_t k = c; k < n; k += nchunk) acc += fabs(w[k]);
  part[c] = acc;
}

// Strided partial sums: slot c adds x[c], x[c + nchunk], ... (coalesced, and a fixed order for a
// given nchunk, so the total is reproducible).
__global__ __launch_bounds__(FT) void k_sum_partial(const double* x, int64_t n, double* part,
                                                    int64_t nchunk) {
  int64_t c = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (c >= nchunk) return;
  double acc = 0.0;
  for (int64_t k = c; k < n; k += nchunk) acc += x[k];
  part[c] = acc;
}

__global__ void k_combine_obj(const double* ll, const double* pen, double lambda, double* out) {
  *out = *ll - lambda * *pen;
}

// ---- W table ----
__global__ void k_winsert(WTable W, int64_t n, const int32_t* ei, const int32_t* ej,
                          const double* w, int64_t N, int directed, int32_t* err) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int i = ei[e], j = ej[e];
  double v = w[e];
  if (i < 0 || j < 0 || i >= N || j >= N || i == j || !isfinite(v)) { atomicOr(err, 8); return; }
  if (v == 0.0) return;
  bool ins;
  const uint64_t key = rec_pair_key(i, j, directed);
  int64_t s = rec_hash_insert(W.keys, W.mask, key, REC_MAX_PROBE, &ins);
  if (s < 0) { atomicOr(err, 2); return; }
  rec_wbloom_set(W, key);
  W.vals[s] = v;
}

// occupied, nonzero table entries -> sort records (key = pair key, val = slot).
// A block takes WC_PER * 256 slots (thread t: slots t, t + 256, ...), counts
// its entries, and reserves one output run with a single atomic.
constexpr int WC_PER = 16;
__global__ __launch_bounds__(256) void k_wcompact(WTable W, uint64_t cap, uint64_t* klo,
                                                  uint32_t* val, int64_t* n, int64_t max_n) {
  __shared__ long long sh[256 / REC_WAVE + 1];
  const uint64_t base = (uint64_t)blockIdx.x * (256 * WC_PER) + threadIdx.x;
  uint32_t keep = 0;
#pragma unroll
  for (int u = 0; u < WC_PER; ++u) {
    const uint64_t s = base + 256u * u;
    if (s < cap && W.keys[s] != REC_EMPTY && W.vals[s] != 0.0) keep |= 1u << u;
  }
  // exclusive prefix of the per-thread counts over the block
  const int lane = threadIdx.x & (REC_WAVE - 1), wave = threadIdx.x / REC_WAVE;
  const int cnt = __popc(keep);
  int inc = cnt;
#pragma unroll
  for (int o = 1; o < REC_WAVE; o <<= 1) {
    const int v = __shfl_up(inc, o, REC_WAVE);
    if (lane >= o) inc += v;
  }
  if (lane == REC_WAVE - 1) sh[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int w = 0; w < 256 / REC_WAVE; ++w) { const long long c = sh[w]; sh[w] = tot; tot += c; }
    sh[256 / REC_WAVE] = tot ? (long long)atomicAdd((unsigned long long*)n, (unsigned long long)tot) : 0;
  }
  __syncthreads();
  int64_t p = (int64_t)(sh[256 / REC_WAVE] + sh[wave]) + (inc - cnt);
  for (uint32_t k = keep; k; k &= k - 1, ++p) {
    const uint64_t s = base + 256u * (uint32_t)__builtin_ctz(k);
    if (p < max_n) { klo[p] = W.keys[s]; val[p] = (uint32_t)s; }
  }
}

__global__ void k_wunpack(const uint64_t* klo, const uint32_t* val, const double* wvals, int64_t n,
                          int32_t* wi, int32_t* wj, double* wv) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  wi[e] = (int32_t)(klo[e] >> 32);
  wj[e] = (int32_t)(klo[e] & 0xffffffffu);
  wv[e] = wvals[val[e]];
}

// CSR records: one per (row, col) direction
__global__ void k_csr_records(const int32_t* wi, const int32_t* wj, int64_t n, int directed,
                              uint64_t* klo, uint32_t* val, int64_t* rowcnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int i = wi[e], j = wj[e];
  if (directed) {
    klo[e] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)j;
    val[e] = (uint32_t)e;
    atomicAdd((unsigned long long*)&rowcnt[i], 1ULL);
  } else {
    klo[2 * e] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)j;
    val[2 * e] = (uint32_t)e;
    klo[2 * e + 1] = ((uint64_t)(uint32_t)j << 32) | (uint32_t)i;
    val[2 * e + 1] = (uint32_t)e;
    atomicAdd((unsigned long long*)&rowcnt[i], 1ULL);
    atomicAdd((unsigned long long*)&rowcnt[j], 1ULL);
  }
}

__global__ void k_csr_fill(const uint64_t* klo, const uint32_t* val, const double* wv, int64_t n,
                           int32_t* col, double* colw) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  col[e] = (int32_t)(klo[e] & 0xffffffffu);
  colw[e] = wv[val[e]];
}

int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) < v) ++b;
  return b < 1 ? 1 : b;
}

template <class R, int NPL>
rec_status launch_fields_n(rec_ctx* ctx) {
  dim3 g((unsigned)((ctx->cfg.N + FT / REC_WAVE - 1) / (FT / REC_WAVE))), b(FT);
  switch (ctx->cfg.model) {
    case REC_ISING:
      hipLaunchKernelGGL((k_fields<R, NPL, REC_ISING>), g, b, 0, ctx->stream, ctx->F, ctx->row_off, ctx->col, ctx->colw);
      break;
    case REC_GAUSS:
      hipLaunchKernelGGL((k_fields<R, NPL, REC_GAUSS>), g, b, 0, ctx->stream, ctx->F, ctx->row_off, ctx->col, ctx->colw);
      break;
    default:
      hipLaunchKernelGGL((k_fields<R, NPL, REC_KINETIC>), g, b, 0, ctx->stream, ctx->F, ctx->row_off, ctx->col, ctx->colw);
  }
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R, int NPL>
rec_status launch_theta_k(rec_ctx* ctx, bool rebuild) {
  dim3 g((unsigned)((ctx->cfg.N + FT / REC_WAVE - 1) / (FT / REC_WAVE))), b(FT);
  const int64_t* ro = rebuild ? ctx->row_off : nullptr;
  switch (ctx->cfg.model) {
    case REC_ISING:
      hipLaunchKernelGGL((k_theta<R, NPL, REC_ISING>), g, b, 0, ctx->stream, ctx->F, ro, ctx->col, ctx->colw);
      break;
    case REC_GAUSS:
      hipLaunchKernelGGL((k_theta<R, NPL, REC_GAUSS>), g, b, 0, ctx->stream, ctx->F, ro, ctx->col, ctx->colw);
      break;
    default:
      hipLaunchKernelGGL((k_theta<R, NPL, REC_KINETIC>), g, b, 0, ctx->stream, ctx->F, ro, ctx->col, ctx->colw);
  }
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R, int NPL>
rec_status launch_theta_n(rec_ctx* ctx) { return launch_theta_k<R, NPL>(ctx, false); }

template <class R, int NPL>
rec_status launch_fields_theta_n(rec_ctx* ctx) { return launch_theta_k<R, NPL>(ctx, true); }

// the row kernels keep NPL samples per lane in registers
#define REC_NPL_SWITCH(FN, R)                                   \
  switch (ctx->F.npl) {                                         \
    case 1: return FN<R, 1>(ctx);                               \
    case 2: return FN<R, 2>(ctx);                               \
    case 4: return FN<R, 4>(ctx);                               \
    case 8: return FN<R, 8>(ctx);                               \
    case 16: return FN<R, 16>(ctx);                             \
    case 32: return FN<R, 32>(ctx);                             \
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL; \
  }

template <class R>
rec_status launch_fields_r(rec_ctx* ctx) { REC_NPL_SWITCH(launch_fields_n, R) }

template <class R>
rec_status launch_theta_r(rec_ctx* ctx) { REC_NPL_SWITCH(launch_theta_n, R) }

template <class R>
rec_status launch_fields_theta_r(rec_ctx* ctx) { REC_NPL_SWITCH(launch_fields_theta_n, R) }

template <class R, int NPL>
rec_status launch_rowll_n(rec_ctx* ctx) {
  dim3 g((unsigned)((ctx->cfg.N + FT / REC_WAVE - 1) / (FT / REC_WAVE))), b(FT);
  switch (ctx->cfg.model) {
    case REC_ISING: hipLaunchKernelGGL((k_rowll<R, NPL, REC_ISING>), g, b, 0, ctx->stream, ctx->F, ctx->dscratch); break;
    case REC_GAUSS: hipLaunchKernelGGL((k_rowll<R, NPL, REC_GAUSS>), g, b, 0, ctx->stream, ctx->F, ctx->dscratch); break;
    default: hipLaunchKernelGGL((k_rowll<R, NPL, REC_KINETIC>), g, b, 0, ctx->stream, ctx->F, ctx->dscratch);
  }
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R>
rec_status launch_rowll_r(rec_ctx* ctx) { REC_NPL_SWITCH(launch_rowll_n, R) }

}  // namespace

rec_status rec_load_data(rec_ctx* ctx, const void* X, int64_t ldx) {
  const int64_t N = ctx->cfg.N;
  if (ctx->cfg.model == REC_GAUSS) {
    hipLaunchKernelGGL(k_load_f32, dim3(N), dim3(FT), 0, ctx->stream, (const float*)X, ldx,
                       ctx->F.M, ctx->F.Mp, (float*)ctx->F.xf, (double*)ctx->F.sq, ctx->err_flag);
  } else {
    hipLaunchKernelGGL(k_load_int8, dim3(N), dim3(FT), 0, ctx->stream, (const int8_t*)X, ldx,
                       ctx->F.M, ctx->F.Mp, ctx->cfg.model == REC_KINETIC ? 1 : 0,
                       (int8_t*)ctx->F.xs, (int8_t*)ctx->F.ys, ctx->err_flag);
    hipLaunchKernelGGL(k_pack_bits, dim3(N), dim3(REC_WAVE), 0, ctx->stream, ctx->F.xs, ctx->F.Mp,
                       ctx->F.npl, const_cast<void*>(ctx->F.xq));
    if (ctx->cfg.model == REC_KINETIC)
      hipLaunchKernelGGL(k_pack_bits, dim3(N), dim3(REC_WAVE), 0, ctx->stream, ctx->F.ys, ctx->F.Mp,
                         ctx->F.npl, const_cast<void*>(ctx->F.yq));
    // zero tail rows of the contraction's operands
    const size_t tail = (size_t)(REC_TAIL_ROWS * ctx->F.Mp);
    REC_HIP(hipMemsetAsync(const_cast<int8_t*>(ctx->F.xs) + N * ctx->F.Mp, 0, tail, ctx->stream));
    REC_HIP(hipMemsetAsync(ctx->F.rq + N * ctx->F.Mp, 0, tail, ctx->stream));
  }
  REC_HIP(hipGetLastError());
  return REC_OK;
}

void rec_wtable_clear(rec_ctx* ctx) {
  ++ctx->w_version;
  ctx->w_any = false;
  hipMemsetAsync(ctx->W.keys, 0xff, (ctx->W.mask + 1) * sizeof(uint64_t), ctx->stream);
  hipMemsetAsync(ctx->W.bloom, 0, REC_WBLOOM_WORDS * sizeof(uint32_t), ctx->stream);
}

rec_status rec_wtable_insert_list(rec_ctx* ctx, int64_t n, const int32_t* ei, const int32_t* ej,
                                  const double* w) {
  if (n <= 0) return REC_OK;
  ++ctx->w_version;
  ctx->w_any = true;
  hipLaunchKernelGGL(k_winsert, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->W, n, ei, ej,
                     w, ctx->cfg.N, ctx->cfg.model == REC_KINETIC ? 1 : 0, ctx->err_flag);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

// Sorted list of nonzero W entries into wi/wj/wv, then the row lists.
rec_status rec_wtable_compact(rec_ctx* ctx, int64_t* nnz_out) {
  if (ctx->w_compacted == ctx->w_version) {
    *nnz_out = ctx->w_nnz;
    return REC_OK;
  }
  const uint64_t cap = ctx->W.mask + 1;
  int64_t* d_n = ctx->counter + 4;
  REC_HIP(hipMemsetAsync(d_n, 0, sizeof(int64_t), ctx->stream));
  hipLaunchKernelGGL(k_wcompact, dim3((cap + 256 * WC_PER - 1) / (256 * WC_PER)), dim3(256), 0, ctx->stream, ctx->W, cap,
                     ctx->sb.klo[0], ctx->sb.val[0], d_n, ctx->max_nnz);
  int64_t n = 0;
  REC_HIP(hipMemcpyAsync(&n, d_n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  if (n > ctx->max_nnz) {
    ctx->err = "more nonzero couplings than max_nnz";
    return REC_E_NOMEM;
  }
  const int nb = bits_for(ctx->cfg.N);
  Digit dg[8];
  int nd = 0;
  for (int s = 0; s < nb; s += 8) dg[nd++] = {0, s};
  for (int s = 0; s < nb; s += 8) dg[nd++] = {0, 32 + s};
  int cur = 0;
  rec_status st = rec_radix_sort(ctx, n, dg, nd, &cur);
  if (st != REC_OK) return st;
  if (n > 0)
    hipLaunchKernelGGL(k_wunpack, dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       ctx->sb.klo[cur], ctx->sb.val[cur], ctx->W.vals, n, ctx->wi, ctx->wj, ctx->wv);
  // row lists: both directions for symmetric models
  const int directed = ctx->cfg.model == REC_KINETIC;
  int64_t nrec = directed ? n : 2 * n;
  REC_HIP(hipMemsetAsync(ctx->cnt, 0, sizeof(int64_t) * (ctx->cfg.N + 1), ctx->stream));
  if (n > 0)
    hipLaunchKernelGGL(k_csr_records, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ctx->wi,
                       ctx->wj, n, directed, ctx->sb.klo[0], ctx->sb.val[0], ctx->cnt);
  cur = 0;
  if (!directed) {   // directed records are the (i, j)-sorted list itself
    st = rec_radix_sort(ctx, nrec, dg, nd, &cur);
    if (st != REC_OK) return st;
  }
  st = rec_exclusive_scan(ctx, ctx->cnt, ctx->row_off, ctx->cfg.N + 1, nullptr);
  if (st != REC_OK) return st;
  if (nrec > 0)
    hipLaunchKernelGGL(k_csr_fill, dim3((nrec + 255) / 256), dim3(256), 0, ctx->stream,
                       ctx->sb.klo[cur], ctx->sb.val[cur], ctx->wv, nrec, ctx->col, ctx->colw);
  REC_HIP(hipGetLastError());
  ctx->w_compacted = ctx->w_version;
  ctx->w_nnz = n;
  *nnz_out = n;
  return REC_OK;
}

rec_status rec_rebuild_fields(rec_ctx* ctx) {
  int64_t nnz;
  rec_status st = rec_wtable_compact(ctx, &nnz);
  if (st != REC_OK) return st;
  return ctx->fp32 ? launch_fields_r<float>(ctx) : launch_fields_r<double>(ctx);
}

rec_status rec_fit_theta(rec_ctx* ctx) {
  return ctx->fp32 ? launch_theta_r<float>(ctx) : launch_theta_r<double>(ctx);
}

rec_status rec_rebuild_fields_fit_theta(rec_ctx* ctx) {
  int64_t nnz;
  rec_status st = rec_wtable_compact(ctx, &nnz);
  if (st != REC_OK) return st;
  return ctx->fp32 ? launch_fields_theta_r<float>(ctx) : launch_fields_theta_r<double>(ctx);
}

rec_status rec_sum_device(rec_ctx* ctx, const double* x, int64_t n, double* out) {
  const int64_t nchunk = std::min<int64_t>(std::max<int64_t>(ctx->cfg.N, 1024),
                                           std::max<int64_t>(1024, (n + 255) / 256));
  hipLaunchKernelGGL(k_sum_partial, dim3((unsigned)((nchunk + FT - 1) / FT)), dim3(FT), 0, ctx->stream, x, n,
                     ctx->dscratch, nchunk);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(FT), 0, ctx->stream, ctx->dscratch, nchunk, out);
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_eval_objective(rec_ctx* ctx, double* out) {
  rec_status st = ctx->fp32 ? launch_rowll_r<float>(ctx) : launch_rowll_r<double>(ctx);
  if (st != REC_OK) return st;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(FT), 0, ctx->stream, ctx->dscratch, ctx->cfg.N,
                     ctx->dresult + 0);
  // penalty over the sorted W list (wi/wj/wv are current after a compaction)
  int64_t nnz;
  st = rec_wtable_compact(ctx, &nnz);
  if (st != REC_OK) return st;
  // about 256 couplings per partial, at most one partial per dscratch slot
  const int64_t nchunk = std::min<int64_t>(std::max<int64_t>(ctx->cfg.N, 1024),
                                           std::max<int64_t>(1024, (nnz + 255) / 256));
  hipLaunchKernelGGL(k_abs_partial, dim3((unsigned)((nchunk + FT - 1) / FT)), dim3(FT), 0, ctx->stream, ctx->wv,
                     nnz, ctx->dscratch, nchunk);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(FT), 0, ctx->stream, ctx->dscratch, nchunk,
                     ctx->dresult + 1);
  hipLaunchKernelGGL(k_combine_obj, dim3(1), dim3(1), 0, ctx->stream, ctx->dresult + 0,
                     ctx->dresult + 1, ctx->cfg.lambda, ctx->dresult + 2);
  REC_HIP(hipMemcpyAsync(out, ctx->dresult + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  REC_HIP(hipStreamSynchronize(ctx->stream));
  REC_HIP(hipGetLastError());
  return REC_OK;
}
