// Exact pair scores [Alg. 2, function D] and coordinate updates [Alg. 2 loop
// body] on gfx950.
//
// One 64-lane wavefront owns one pair at a time; its lanes split the M
// samples (lane l holds samples c*64*VEC + l*VEC + k, so every load
// instruction of the wave reads one contiguous block).  The j-side row is
// read once into registers and every Newton step afterwards is register
// only; consecutive pairs with the same i keep the i-side row.
//
// Ising / kinetic score.  For x in {-1, 0, 1} (0 = padding) and t = tanh h,
//   x tanh(h + delta x) = (u + tau) / (1 + u tau),   u = x t,  tau = tanh delta
// (tanh addition formula), and
//   log cosh(h + delta x) - log cosh h = log cosh delta + log(1 + u tau).
// So the derivative of the smooth part of the objective change,
//   Phi(tau) = c S - sum_m y_m,  y_m = (u_m + tau) / (1 + u_m tau),
// costs one reciprocal per sample and side, and the gain at the root is
//   c delta S - n M log cosh delta - sum log(1 + u tau) - lambda (|w| - |w0|)
// (c = n = 2 for the symmetric Ising model, whose pair touches the
// conditionals of i and j [App. A]; c = n = 1 for the kinetic model, where
// only row i's conditional depends on W_ij).  Phi is decreasing in tau, and
// the L1 kink sits at tau0 = tanh(-w0) (w = 0): if |Phi(tau0)| <= lambda the
// optimum is w = 0, else the root of Phi = s lambda (s = sign Phi(tau0))
// lies in (tau0, 1) or (-1, tau0); Newton steps inside that bracket,
// bisection otherwise.  dPhi/dtau uses 1 - y^2 = (1 - u^2)(1 - tau^2)/(1 + u tau)^2.
//
// Start of the search at w0 = 0 (every candidate not yet in W): at tau = 0,
// y = u, so Phi(0) = c S - sum u and dPhi/dtau(0) = -sum (1 - u^2) come from
// the load itself with no reciprocal; below the L1 threshold the pair is done.
// Otherwise (u + tau)/(1 + u tau) = u + (1 - u^2) tau (1 - u tau + u^2 tau^2 ...)
// gives Phi(tau) = Phi(0) - mu0 tau + mu1 tau^2 - mu2 tau^3 + mu3 tau^4 + ...
// with mu_k = sum (1 - u^2) u^k; the root of that quartic starts Newton, which
// then usually confirms convergence after one full evaluation.
//
// Kinetic search score: FindBest needs a symmetric score, so inside it the
// unordered pair {i, j} of the kinetic model is scored by the larger of the
// gains of W_ij and W_ji.  One wave loads both nodes' rows once and runs the
// two one-sided solves (u = x_j t_i against targets y_i, v = x_i t_j against
// y_j) back to back.
//
// Gaussian score: closed form.  With residuals r_i = x_i + theta_i^2 m_i the
// change of the two conditionals [App. A] is a delta - b delta^2 / 2 with
// a = -(r_i . x_j + r_j . x_i), b = theta_i^2 |x_j|^2 + theta_j^2 |x_i|^2,
// maximised with the L1 term by soft thresholding.
#include <algorithm>
#include <math.h>

#include "common.hpp"
#include "ctx.hpp"

namespace {

// the kinetic model's symmetrised search score (internal model tag)
constexpr int REC_KINSYM = 3;

template <class R> struct Prec;
template <> struct Prec<float> {
  static constexpr double tol = 3e-5;   // next Newton error ~ tol^2, below float noise
  static constexpr int maxit = 24;
};
template <> struct Prec<double> {
  static constexpr double tol = 1e-12;
  static constexpr int maxit = 60;
};

__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float tanh_(float x) { return tanhf(x); }
__device__ __forceinline__ double tanh_(double x) { return tanh(x); }
__device__ __forceinline__ float log_(float x) { return __logf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }

// load VEC int8 samples as floats
template <int VEC>
__device__ __forceinline__ void ld_x(const int8_t* p, float* o) {
  if constexpr (VEC == 4) {
    int v = *reinterpret_cast<const int*>(p);
    o[0] = (float)(int8_t)(v & 0xff);
    o[1] = (float)(int8_t)((v >> 8) & 0xff);
    o[2] = (float)(int8_t)((v >> 16) & 0xff);
    o[3] = (float)(int8_t)((v >> 24) & 0xff);
  } else if constexpr (VEC == 2) {
    short v = *reinterpret_cast<const short*>(p);
    o[0] = (float)(int8_t)(v & 0xff);
    o[1] = (float)(int8_t)((v >> 8) & 0xff);
  } else {
    o[0] = (float)p[0];
  }
}

template <int VEC, class R>
__device__ __forceinline__ void ld_r(const R* p, R* o) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) o[k] = p[k];
}

template <int VEC>
__device__ __forceinline__ void ld_f(const float* p, float* o) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) o[k] = p[k];
}

// offset of this lane's k-th sample of chunk c
template <int VEC>
__device__ __forceinline__ int64_t smp(int c, int lane) {
  return (int64_t)c * (REC_WAVE * VEC) + (int64_t)lane * VEC;
}

__device__ __forceinline__ double lookup_w(const WTable& W, int i, int j, bool directed) {
  if (W.keys == nullptr) return 0.0;
  const uint64_t key = rec_pair_key(i, j, directed);
  if (!rec_wbloom_maybe(W, key)) return 0.0;   // never inserted
  int64_t s = rec_hash_find(W.keys, W.mask, key, REC_MAX_PROBE);
  return s < 0 ? 0.0 : W.vals[s];
}

// Per-pair registers of one lane.
template <class R, int NPL>
struct Lane {
  static constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  R ti[NPL];      // i side: tanh h_i (Ising / kinetic); r_i (Gaussian)
  R xi[NPL];      // i side: x_i (symmetric) or target y_i (kinetic)
  R u[NPL];       // x_j t_i (Ising / kinetic); x_j (Gaussian)
  R v[NPL];       // x_i t_j (Ising, kinetic search); r_j (Gaussian)
  int xin[CH];    // kinetic search: input-side samples x_i, VEC bytes per chunk
};

// Raw j-side row of one lane, loaded ahead of its use.
template <class R, int NPL, int MODEL>
struct JRaw {
  static constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  int xb[CH];                                      // VEC int8 samples per chunk
  R t[MODEL == REC_KINETIC ? 1 : NPL];             // t_j (Ising) or r_j (Gaussian)
  float xg[MODEL == REC_GAUSS ? NPL : 1];          // x_j (Gaussian)
};

template <int VEC>
__device__ __forceinline__ int ld_bytes(const int8_t* p) {
  if constexpr (VEC == 4) return *reinterpret_cast<const int*>(p);
  else if constexpr (VEC == 2) return (int)*reinterpret_cast<const unsigned short*>(p);
  else return (int)(unsigned char)p[0];
}
__device__ __forceinline__ float byte_at(int w, int k) { return (float)(int8_t)((w >> (8 * k)) & 0xff); }

template <int VEC, class R>
__device__ __forceinline__ void ld_vec(const R* p, R* o) {
  if constexpr (VEC == 4 && sizeof(R) == 4) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if constexpr (VEC == 4 && sizeof(R) == 8) {
    double2 a = *reinterpret_cast<const double2*>(p);
    double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) o[k] = p[k];
  }
}

template <class R, int NPL, int MODEL>
__device__ __forceinline__ void fetch_j(const Fields& F, int j, JRaw<R, NPL, MODEL>& r, int lane) {
  constexpr int VEC = JRaw<R, NPL, MODEL>::VEC, CH = JRaw<R, NPL, MODEL>::CH;
  const int64_t row = (int64_t)j * F.Mp;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    int64_t o = smp<VEC>(c, lane);
    if constexpr (MODEL == REC_GAUSS) {
      ld_vec<VEC>(F.xf + row + o, r.xg + c * VEC);
      ld_vec<VEC>(reinterpret_cast<const R*>(F.H) + row + o, r.t + c * VEC);
    } else {
      r.xb[c] = ld_bytes<VEC>(F.xs + row + o);
      if constexpr (MODEL == REC_ISING) ld_vec<VEC>(reinterpret_cast<const R*>(F.T) + row + o, r.t + c * VEC);
    }
  }
}

// sum over the lane's samples of y = (a + tau)/(1 + a tau) and y^2
template <class R, int NPL>
__device__ __forceinline__ void side_sums(const R* a, R tau, R& A, R& Q) {
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    R d = fma(a[k], tau, R(1));
    R r = rcp_(d);
    R y = (a[k] + tau) * r;
    A += y;
    Q = fma(y, y, Q);
  }
}

// sum over the lane's samples of log(1 + a tau), by products of 4 factors
template <class R, int NPL>
__device__ __forceinline__ double side_logs(const R* a, R tau) {
  double L = 0.0;
#pragma unroll
  for (int k0 = 0; k0 < NPL; k0 += 4) {
    R prod = R(1);
#pragma unroll
    for (int k = k0; k < k0 + 4 && k < NPL; ++k) prod *= fma(a[k], tau, R(1));
    L += (double)log_(prod);
  }
  return L;
}

struct PairOut { double gain, w, w0; };

// Work counters of one wave: pairs, moment passes, full Newton evaluations,
// log passes, sides decided by the residual screen, j-side tanh rows fetched,
// i-side row loads, and the algorithmic bytes read and written (the data the
// method needs per unit, not cache-line traffic): per pair its indices, cache
// slot and score; per j-side read the bytes of the rows it fetches; per i
// row load that row's data, all at M samples.
struct Work {
  int64_t pairs = 0, moments = 0, evals = 0, logs = 0, screened = 0, tfetch = 0, iloads = 0;
  int64_t bytes = 0;
  __device__ void flush(int64_t* work, int64_t wave) const {
    int64_t* wc = work + REC_WORK_N * (wave & (REC_WORK_COPIES - 1));
    const int64_t v[8] = {pairs, moments, evals, logs, screened, tfetch, iloads, bytes};
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (v[q]) atomicAdd((unsigned long long*)&wc[q], (unsigned long long)v[q]);
  }
};

// Ising / kinetic: u (and v) into the lane registers; returns this lane's part
// of Phi(0) = c S - sum u (- sum v) and its part of S in *s_lane.
template <class R, int NPL, int MODEL>
__device__ __forceinline__ double form_j(const JRaw<R, NPL, MODEL>& r, Lane<R, NPL>& L,
                                         float* s_lane) {
  constexpr int VEC = JRaw<R, NPL, MODEL>::VEC, CH = JRaw<R, NPL, MODEL>::CH;
  float s = 0.f;
  R a = R(0), a2 = R(0);
#pragma unroll
  for (int c = 0; c < CH; ++c) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const int q = c * VEC + k;
      if constexpr (MODEL == REC_GAUSS) {
        L.u[q] = (R)r.xg[q];
        L.v[q] = r.t[q];
      } else {
        float x = byte_at(r.xb[c], k);
        R u = (R)x * L.ti[q];
        L.u[q] = u;
        a += u;
        if constexpr (MODEL == REC_ISING) {
          R v = L.xi[q] * r.t[q];
          L.v[q] = v;
          a2 += v;
        }
        s += x * (float)L.xi[q];      // +-1 products: exact in float
      }
    }
  }
  *s_lane = s;
  constexpr double c = MODEL == REC_ISING ? 2.0 : 1.0;
  return c * (double)s - ((double)a + (double)a2);
}

// Exact score of pair (i, j) for the Ising (TWO = true) or kinetic model,
// with u (and v) the lane's sample terms; phi0 = Phi(0) (uniform); s_lane =
// this lane's part of S.
template <class R, int NPL, bool TWO>
__device__ __forceinline__ PairOut solve_ising(const R (&Lu)[NPL], const R (&Lv)[NPL], double phi0,
                                               float s_lane, double w0, double lambda, int64_t M,
                                               int64_t Mp, Work& wk) {
  constexpr double nsides = TWO ? 2.0 : 1.0;
  constexpr double c = TWO ? 2.0 : 1.0;
  const double npad = (double)(Mp - M);
  PairOut o;
  o.w0 = w0;
  if (w0 == 0.0 && fabs(phi0) <= lambda) { o.gain = 0.0; o.w = 0.0; return o; }
  const double Sc = c * (double)rec_wave_sum_dpp((int)s_lane);
  auto eval = [&](double tau, double& phi, double& dphi) {
    // the two sides are summed apart and added once, so (i,j) and (j,i) give
    // the same bits
    R A = R(0), Q = R(0), A2 = R(0), Q2 = R(0);
    side_sums<R, NPL>(Lu, (R)tau, A, Q);
    if constexpr (TWO) side_sums<R, NPL>(Lv, (R)tau, A2, Q2);
    double As = rec_wave_sum_dpp((double)A + (double)A2);
    double Qs = rec_wave_sum_dpp((double)Q + (double)Q2);
    double t = (double)(R)tau;
    phi = Sc - As + nsides * npad * t;
    double om = 1.0 - t * t;
    dphi = -((nsides * (double)Mp - Qs) / om - nsides * npad);
    ++wk.evals;
  };
  double tau0, phi, dphi;
  double mu1 = 0.0, mu2 = 0.0, mu3 = 0.0;
  if (w0 == 0.0) {
    // moments mu_k = sum (1 - u^2) u^k; padding has u = 0, so only mu0 sees it
    R m0 = R(0), m1 = R(0), m2 = R(0), m3 = R(0), n0 = R(0), n1 = R(0), n2 = R(0), n3 = R(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      R u = Lu[k];
      R q = fma(-u, u, R(1));
      m0 += q;
      R t1 = q * u;
      m1 += t1;
      R t2 = t1 * u;
      m2 += t2;
      m3 = fma(t2, u, m3);
      if constexpr (TWO) {
        R v = Lv[k];
        R qv = fma(-v, v, R(1));
        n0 += qv;
        R s1 = qv * v;
        n1 += s1;
        R s2 = s1 * v;
        n2 += s2;
        n3 = fma(s2, v, n3);
      }
    }
    double mu0 = rec_wave_sum_dpp((double)m0 + (double)n0) - nsides * npad;
    mu1 = rec_wave_sum_dpp((double)m1 + (double)n1);
    mu2 = rec_wave_sum_dpp((double)m2 + (double)n2);
    mu3 = rec_wave_sum_dpp((double)m3 + (double)n3);
    ++wk.moments;
    tau0 = 0.0;
    phi = phi0;
    dphi = -mu0;
  } else {
    tau0 = (double)tanh_((R)(-w0));
    eval(tau0, phi, dphi);
  }
  double tau;
  if (fabs(phi) <= lambda) {
    tau = tau0;     // w0 != 0 here: the optimum is w = 0
    o.w = 0.0;
  } else {
    double s = phi > 0 ? 1.0 : -1.0;
    double target = s * lambda;
    double lo = s > 0 ? tau0 : -1.0, hi = s > 0 ? 1.0 : tau0;
    double f = phi - target, df = dphi;
    tau = tau0;
    if (w0 == 0.0) {
      // root of the quartic model f - mu0 t + mu1 t^2 - mu2 t^3 + mu3 t^4
      const double mu0 = -df;
      double t = f / mu0;
      for (int q = 0; q < 8; ++q) {
        double P = f + t * (-mu0 + t * (mu1 + t * (-mu2 + t * mu3)));
        double dP = -mu0 + t * (2.0 * mu1 + t * (-3.0 * mu2 + t * 4.0 * mu3));
        if (!(dP < 0)) break;
        t -= P / dP;
      }
      if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
      tau = t;
      eval(tau, phi, dphi);
      f = phi - target;
      df = dphi;
    }
    for (int it = 0; it < Prec<R>::maxit; ++it) {
      if (f > 0) lo = tau; else hi = tau;
      double tn = (df < 0) ? tau - f / df : 0.5 * (lo + hi);
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
      double step = tn - tau;
      tau = tn;
      if (fabs(step) <= Prec<R>::tol * fmax(fabs(tau), 1e-4)) break;
      eval(tau, phi, dphi);
      f = phi - target;
      df = dphi;
    }
    tau = (double)(R)tau;
    double d = rec_atanh(tau);
    double w = w0 + d;
    o.w = s > 0 ? fmax(w, 0.0) : fmin(w, 0.0);
  }
  double Ls = side_logs<R, NPL>(Lu, (R)tau);
  if constexpr (TWO) Ls += side_logs<R, NPL>(Lv, (R)tau);
  Ls = rec_wave_sum_dpp(Ls);
  ++wk.logs;
  double d = rec_atanh(tau);
  double g = Sc * d - nsides * (double)M * rec_lcosh_tau(tau) - Ls -
             lambda * (fabs(o.w) - fabs(w0));
  o.gain = g;
  return o;
}

// Gaussian closed form with u = x_j, v = r_j, ti = r_i, xi = x_i in the lane.
template <class R, int NPL>
__device__ PairOut solve_gauss(const Lane<R, NPL>& L, double vi, double vj, double sqi, double sqj,
                               double w0, double lambda) {
  R a = R(0);
#pragma unroll
  for (int k = 0; k < NPL; ++k) a = fma(L.ti[k], L.u[k], fma(L.v[k], L.xi[k], a));
  double as = -rec_wave_sum_dpp((double)a);
  double b = vi * sqj + vj * sqi;
  double z = w0 + as / b;
  double ws = z > 0 ? fmax(z - lambda / b, 0.0) : fmin(z + lambda / b, 0.0);
  double d = ws - w0;
  PairOut o;
  o.w0 = w0;
  o.w = ws;
  o.gain = as * d - 0.5 * b * d * d - lambda * (fabs(ws) - fabs(w0));
  return o;
}

// Load the i-side registers of node i.
template <class R, int NPL, int MODEL>
__device__ __forceinline__ void load_i(const Fields& F, int i, Lane<R, NPL>& L, int lane) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const R* Hr = reinterpret_cast<const R*>(MODEL == REC_GAUSS ? F.H : F.T) + (int64_t)i * F.Mp;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    int64_t o = smp<VEC>(c, lane);
    ld_vec<VEC>(Hr + o, L.ti + c * VEC);
    if constexpr (MODEL == REC_GAUSS) {
      float xv[VEC];
      ld_vec<VEC>(F.xf + (int64_t)i * F.Mp + o, xv);
#pragma unroll
      for (int k = 0; k < VEC; ++k) L.xi[c * VEC + k] = (R)xv[k];
    } else {
      constexpr bool kin = MODEL == REC_KINETIC || MODEL == REC_KINSYM;
      int w = ld_bytes<VEC>((kin ? F.ys : F.xs) + (int64_t)i * F.Mp + o);
#pragma unroll
      for (int k = 0; k < VEC; ++k) L.xi[c * VEC + k] = (R)byte_at(w, k);
      if constexpr (MODEL == REC_KINSYM) L.xin[c] = ld_bytes<VEC>(F.xs + (int64_t)i * F.Mp + o);
    }
  }
}

template <class R, int NPL, int MODEL>
__device__ __forceinline__ PairOut solve(const Fields& F, const Lane<R, NPL>& L, double phi0,
                                         float s_lane, int i, int j, double w0, double lambda,
                                         Work& wk) {
  ++wk.pairs;
  if constexpr (MODEL == REC_GAUSS) {
    double vi = F.theta[i] * F.theta[i], vj = F.theta[j] * F.theta[j];
    return solve_gauss<R, NPL>(L, vi, vj, F.sq[i], F.sq[j], w0, lambda);
  } else {
    return solve_ising<R, NPL, MODEL == REC_ISING>(L.u, L.v, phi0, s_lane, w0, lambda, F.M, F.Mp, wk);
  }
}

// 0 <= i, j < N (N < 2^31) and i != j, in 32-bit scalar compares
__device__ __forceinline__ bool pair_ok(int i, int j, int64_t N) {
  const uint32_t n = (uint32_t)N;
  return (uint32_t)i < n && (uint32_t)j < n && i != j;
}

constexpr int SKIP = -2;   // pair not owned by this launch (owner mode)
constexpr uint32_t OWNER = 0x80000000u;

// Pairs (I[p], J[p]) (J through Smap when given).  slot == null: results to
// gain_out[p]; otherwise to the cache slot slot[p] (owner mode: only entries
// whose slot word has the owner bit are scored).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) void k_score(Fields F, WTable W, double lambda, int64_t P,
                                               const int32_t* __restrict__ I,
                                               const int32_t* __restrict__ J,
                                               const int32_t* __restrict__ Smap,
                                               const uint32_t* __restrict__ slot, int owned,
                                               double* __restrict__ gain_out,
                                               double* __restrict__ w_out, double* __restrict__ ovf,
                                               uint64_t cache_cap, int32_t* err, int ppw,
                                               int64_t* work) {
  const int lane = rec_lane();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE;
  int64_t p0 = wave * ppw;
  if (p0 >= P) return;
  int np = (int)(p0 + ppw < P ? ppw : P - p0);
  // lanes 0..np-1 fetch the pairs of this wave and their current weights at once
  int li = -1, lj = -1;
  double lw = 0.0;
  if (lane < np) {
    uint32_t sw = slot ? slot[p0 + lane] : 0u;
    if (owned && !(sw & OWNER)) {
      li = SKIP;
    } else {
      li = I[p0 + lane];
      lj = J[p0 + lane];
      if (Smap) lj = Smap[lj];
      if (pair_ok(li, lj, F.N)) lw = lookup_w(W, li, lj, MODEL == REC_KINETIC);
    }
  }
  Lane<R, NPL> L;
  JRaw<R, NPL, MODEL> nx;
  int cur = -1;
  Work wk;
  // the pairs this wave scores, in order: one bit per lane holding one
  uint64_t todo = __ballot(lane < np && li != SKIP);
  if (todo) {
    int q0 = __ffsll((unsigned long long)todo) - 1;
    int i0 = rec_lane_val(li, q0), j0 = rec_lane_val(lj, q0);
    if (pair_ok(i0, j0, F.N)) fetch_j<R, NPL, MODEL>(F, j0, nx, lane);
  }
  while (todo) {
    const int q = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const int64_t p = p0 + q;
    int i = rec_lane_val(li, q), j = rec_lane_val(lj, q);
    double w0 = rec_lane_val(lw, q);
    JRaw<R, NPL, MODEL> rw = nx;   // holds this pair's row (fetched ahead)
    if (todo) {                    // next pair's row in flight while this one computes
      const int q1 = __ffsll((unsigned long long)todo) - 1;
      int i1 = rec_lane_val(li, q1), j1 = rec_lane_val(lj, q1);
      if (pair_ok(i1, j1, F.N)) fetch_j<R, NPL, MODEL>(F, j1, nx, lane);
    }
    double* dst = gain_out + p;
    if (slot) {
      const uint64_t o = (uint64_t)(slot[p] & ~OWNER);
      dst = o >= cache_cap ? ovf + (o - cache_cap) : gain_out + o;
    }
    if (!pair_ok(i, j, F.N)) {
      if (lane == 0) {
        *dst = __builtin_nan("");
        if (w_out) w_out[p] = __builtin_nan("");
        atomicOr(err, 1);
      }
      continue;
    }
    if (i != cur) { load_i<R, NPL, MODEL>(F, i, L, lane); cur = i; ++wk.iloads; }
    ++wk.tfetch;
    float s_lane;
    double phi_l = form_j<R, NPL, MODEL>(rw, L, &s_lane);
    double phi0 = MODEL == REC_GAUSS ? 0.0 : rec_wave_sum_dpp(phi_l);
    PairOut r = solve<R, NPL, MODEL>(F, L, phi0, s_lane, i, j, w0, lambda, wk);
    double g = r.gain;
    if constexpr (sizeof(R) == 4) g = (double)(float)g;   // FP32 scores
    if (lane == 0) {
      *dst = g;
      if (w_out) w_out[p] = r.w;
    }
  }
  if (lane == 0 && work) {
    const int64_t M = F.M, rs = sizeof(R);
    const int64_t jb = MODEL == REC_ISING ? M + rs * M : MODEL == REC_KINETIC ? M : 4 * M + rs * M;
    const int64_t ib = MODEL == REC_GAUSS ? rs * M + 4 * M : rs * M + M;
    wk.bytes = wk.tfetch * (16 + (slot ? 4 : 0) + jb) + wk.iloads * ib;
    wk.flush(work, wave);
  }
}

// ----------------------------------------------------- gradient distance --
// Gradient as distance [Appendix, "Gradient as distance"]: the search scores a
// pair by the absolute derivative of the objective in W_ij at the current
// state, taken as a central difference at the L1 kink: |F'(w0) - lambda
// sign(w0)| for a current coupling, |F'(0)| for a new pair.  F' is one pass
// over the samples (no Newton solve): for row a's conditional,
//   dF_a / dW_ab = sum_m x_b,m r_a,m,  r_a = y_a - tanh h_a   (Ising, kinetic),
//                = -sum_m r_a,m x_b,m,  r_a the residual       (Gaussian),
// summed over both conditionals for the symmetric models; the kinetic search
// over unordered pairs takes the larger of the two directions (as for the
// gain).  Same interface as k_score: pairs (I[p], J[p]) (J through Smap when
// given), results to gain_out[p] or to the cache slot (owner mode: only
// owned entries are scored).  A wavefront takes ppw pairs in order; lane l
// holds the samples c*64*VEC + l*VEC + k of the i side (r_i, x_i) in registers
// and keeps them while consecutive pairs share i, so a pair streams the j
// side only (x_j; with r_j for the symmetric and two-direction scores).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) void k_grad(Fields F, WTable W, double lambda, int64_t P,
                                              const int32_t* __restrict__ I,
                                              const int32_t* __restrict__ J,
                                              const int32_t* __restrict__ Smap,
                                              const uint32_t* __restrict__ slot, int owned,
                                              double* __restrict__ gain_out, double* __restrict__ ovf,
                                              uint64_t cache_cap, int32_t* err, int ppw, int64_t* work) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  constexpr bool GAUSS = MODEL == REC_GAUSS, TWO = MODEL != REC_KINETIC;   // TWO: j side's residual too
  const int lane = rec_lane();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE;
  const int64_t p0 = wave * ppw;
  if (p0 >= P) return;
  const int np = (int)(p0 + ppw < P ? ppw : P - p0);
  const R* T = reinterpret_cast<const R*>(F.T);
  const R* Hr = reinterpret_cast<const R*>(F.H);
  const int8_t* Y = MODEL == REC_ISING ? F.xs : F.ys;
  // row b's residual and inputs at this lane's samples (Gaussian: r = the
  // stored residual with the sign of -F'; x = the float samples)
  auto load_row = [&](int64_t b, double* r, float* x) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t o = b * F.Mp + smp<VEC>(c, lane);
      if constexpr (GAUSS) {
        R h[VEC];
        ld_vec<VEC>(Hr + o, h);
        ld_vec<VEC>(F.xf + o, x + c * VEC);
#pragma unroll
        for (int k = 0; k < VEC; ++k) r[c * VEC + k] = -(double)h[k];
      } else {
        R t[VEC];
        float y[VEC];
        ld_vec<VEC>(T + o, t);
        ld_x<VEC>(Y + o, y);
        ld_x<VEC>(F.xs + o, x + c * VEC);
#pragma unroll
        for (int k = 0; k < VEC; ++k) r[c * VEC + k] = (double)y[k] - (double)t[k];
      }
    }
  };
  auto dot = [&](const double* r, const float* x) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NPL; ++q) acc += (double)x[q] * r[q];
    return rec_wave_sum(acc);
  };
  auto dist = [&](double f1, double w0) {
    return fabs(w0 == 0.0 ? f1 : f1 - lambda * (w0 > 0.0 ? 1.0 : -1.0));
  };
  uint32_t sw = 0u;
  if (lane < np && slot) sw = slot[p0 + lane];
  uint64_t todo = __ballot(lane < np && !(owned && !(sw & OWNER)));
  int64_t pairs = 0, iloads = 0;
  double ri[NPL];
  float xi[NPL];
  int cur = -1;
  while (todo) {
    const int q = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const int64_t p = p0 + q;
    const int i = I[p];
    int j = J[p];
    if (Smap) j = Smap[j];
    const uint64_t o = slot ? (uint64_t)((uint32_t)rec_lane_val((int)sw, q) & ~OWNER) : (uint64_t)p;
    double* dst = (slot && o >= cache_cap) ? ovf + (o - cache_cap) : gain_out + o;
    if (!pair_ok(i, j, F.N)) {
      if (lane == 0) {
        *dst = __builtin_nan("");
        atomicOr(err, 1);
      }
      continue;
    }
    if (i != cur) {
      load_row(i, ri, xi);
      cur = i;
      ++iloads;
    }
    double rj[TWO ? NPL : 1];
    float xj[NPL];
    if constexpr (TWO) {
      load_row(j, rj, xj);
    } else {
#pragma unroll
      for (int c = 0; c < CH; ++c) ld_x<VEC>(F.xs + (int64_t)j * F.Mp + smp<VEC>(c, lane), xj + c * VEC);
    }
    const double dij = dot(ri, xj);   // row i's conditional in W_ij
    double g;
    if constexpr (MODEL == REC_KINETIC) {
      g = dist(dij, lookup_w(W, i, j, true));
    } else if constexpr (MODEL == REC_KINSYM) {
      g = fmax(dist(dij, lookup_w(W, i, j, true)), dist(dot(rj, xi), lookup_w(W, j, i, true)));
    } else {
      g = dist(dij + dot(rj, xi), lookup_w(W, i, j, false));
    }
    if constexpr (sizeof(R) == 4) g = (double)(float)g;   // FP32 scores
    if (lane == 0) *dst = g;
    ++pairs;
  }
  if (lane == 0 && work && pairs) {
    Work wk;
    wk.pairs = pairs;
    wk.iloads = iloads;
    const int64_t M = F.M, rs = sizeof(R);
    const int64_t row = GAUSS ? (rs + 4) * M : (rs + 2) * M;   // a whole row (r and x)
    wk.bytes = pairs * (16 + (TWO ? row : M)) + iloads * row;
    wk.flush(work, wave);
  }
}

// ------------------------------------------------------------ screened --
// Ising and the kinetic search score, with the j side read in two steps.
//
// At w0 = 0 the pair's gain is zero exactly when |Phi(0)| <= lambda (the L1
// kink test).  Phi(0) splits into a part that needs only the signs of x_j
// and the resident i row, and a part sum_m x_i (y_j - t_j) that needs the j
// row's tanh values.  The first read fetches the sign words of x_j (and of
// y_j for the kinetic search) and int8 copies q_j = round(63.5 (y_j - t_j))
// (1.1 bytes per sample instead of 5-6); their error moves the second part by
// at most the bound folded into F.scr, so |screen| <= F.scr proves |Phi(0)| <= lambda
// and the side's gain is exactly zero, the value the full evaluation gives.
// The first part is screened the same way from a resident fp32/fp64 copy of
// r_i (its only error is float rounding, bounded in F.scra).  Otherwise the
// tanh rows are fetched and the side is scored exactly as by k_score: the
// result is the same bits either way.
template <int NPL, bool SYM>
struct JScr {
  static constexpr int UW = rec_u4_words(NPL);
  uint32_t xw;             // signs of x_j (bit q = lane register q)
  uint32_t yw;             // kinetic search: signs of the targets y_j
  uint32_t uw[UW];         // 4-bit copies of 1 - y_j t_j (register q in nibble q % 8 of word q / 8)
};

template <int NPL, bool SYM>
__device__ __forceinline__ void fetch_scr(const Fields& F, int j, JScr<NPL, SYM>& r, int lane) {
  constexpr int UW = JScr<NPL, SYM>::UW;
  // j is wave-uniform: the row bases are scalar and every lane adds a 32-bit
  // offset (no 64-bit lane addresses)
  using ST = rec_sign_t<NPL>;
  r.xw = (uint32_t)(reinterpret_cast<const ST*>(F.xq) + (int64_t)j * REC_WAVE)[lane];
  if constexpr (SYM) r.yw = (uint32_t)(reinterpret_cast<const ST*>(F.yq) + (int64_t)j * REC_WAVE)[lane];
  const uint32_t* ur = F.u4 + (int64_t)j * UW * REC_WAVE;
#pragma unroll
  for (int w = 0; w < UW; ++w) r.uw[w] = ur[w * REC_WAVE + lane];
}

// the int8 copies of y_j - t_j, VEC per word (register c VEC + k in byte k of
// word c), for the sides the 4-bit test leaves open
template <int NPL>
__device__ __forceinline__ void fetch_q8(const Fields& F, int j, uint32_t (&qw)[NPL / (NPL < 4 ? NPL : 4)], int lane) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int8_t* qr = F.rq + (int64_t)j * F.Mp;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const uint32_t o = (uint32_t)(c * REC_WAVE * VEC + lane * VEC);
    if constexpr (VEC == 4) qw[c] = *reinterpret_cast<const uint32_t*>(qr + o);
    else if constexpr (VEC == 2) qw[c] = *reinterpret_cast<const uint16_t*>(qr + o);
    else qw[c] = (uint8_t)qr[o];
  }
}

__device__ __forceinline__ float sgn_at(uint32_t w, int q) { return ((w >> q) & 1u) ? 1.f : -1.f; }
// the int8 copy of register q (exact small integer; scaled once per sum)
template <int NPL, int CH>
__device__ __forceinline__ float q_at(const uint32_t (&qw)[CH], int q) {
  constexpr int VEC = NPL < 4 ? NPL : 4;
  return (float)(int8_t)(qw[q / VEC] >> (8 * (q % VEC)));
}

// the j row of tanh values, fetched only for pairs the screen does not settle
template <class R, int NPL>
__device__ __forceinline__ void fetch_t(const Fields& F, int j, R (&t)[NPL], int lane) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const R* Tr = reinterpret_cast<const R*>(F.T) + (int64_t)j * F.Mp;
#pragma unroll
  for (int c = 0; c < CH; ++c) ld_vec<VEC>(Tr + smp<VEC>(c, lane), t + c * VEC);
}

// The i side of the screened kernels keeps only what the kink tests need in
// registers: the int8 copy q_i of y_i - t_i (zero in the padding) and the
// sign words of the inputs x_i.  Both kink sums are then one select and one
// add per sample, in exact small integers:
//   sum_m x_{j,m} q_{i,m}  (the i <- j part)   and
//   sum_m x_{i,m} q_{j,m}  (the j <- i part),
// each over 63.5, each off the exact residual sum by at most M (1/127 +
// 2^-22) (rec_q8), with padding cancelled by the zeros of q_i and q_j.  The
// exact path (a side whose test does not settle it) reloads t_i and the int8
// rows of i and evaluates the side with the same arithmetic as k_score, so
// its results are the same bits.
// Bits b_0..b_3 of a sign nibble spread to the bytes of a word (byte k = b_k):
// the multiply moves bit k to bit 8k, no two partial products overlap.
__device__ __forceinline__ uint32_t spread01(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }
// The same as +-1 bytes (0x01 for a set bit, 0xFF otherwise): 0xFE times a 0/1
// byte never carries into the next byte.
__device__ __forceinline__ uint32_t spread_pm1(uint32_t nib) { return ~(spread01(nib) * 0xFEu); }

template <class R, int NPL>
struct LaneR {
  static constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC, UW = rec_u4_words(NPL);
  uint32_t ui[UW];   // 4-bit copies of 1 - y_i t_i (as JScr::uw)
  int su;            // sum of the lane's 4-bit copies
  uint32_t qw[CH];   // q_i, VEC bytes per word in the lane layout
  uint32_t pm[CH];   // x_i as +-1 bytes in the same layout (0 past VEC bytes)
  uint32_t xw;       // signs of the inputs x_i (lane word)
  uint32_t yw;       // kinetic search: signs of the targets y_i
  int sq;            // sum of the lane's q_i
};

template <class R, int NPL, int MODEL>
__device__ __forceinline__ void load_i_r(const Fields& F, int i, LaneR<R, NPL>& L, int lane) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int8_t* qr = F.rq + (int64_t)i * F.Mp;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = smp<VEC>(c, lane);
    if constexpr (VEC == 4) L.qw[c] = *reinterpret_cast<const uint32_t*>(qr + o);
    else if constexpr (VEC == 2) L.qw[c] = *reinterpret_cast<const uint16_t*>(qr + o);
    else L.qw[c] = (uint8_t)qr[o];
  }
  L.xw = rec_sign_word<NPL>(F.xq, i, lane);
  L.yw = MODEL == REC_KINSYM ? rec_sign_word<NPL>(F.yq, i, lane) : L.xw;
  L.su = 0;
#pragma unroll
  for (int w = 0; w < LaneR<R, NPL>::UW; ++w) {
    L.ui[w] = F.u4[((int64_t)i * LaneR<R, NPL>::UW + w) * REC_WAVE + lane];
    L.su = (int)__builtin_amdgcn_udot8(L.ui[w], 0x11111111u, (uint32_t)L.su, false);
  }
  L.sq = 0;
  constexpr uint32_t vmask = VEC == 4 ? 0xffffffffu : (1u << (8 * VEC)) - 1u;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    L.pm[c] = spread_pm1((L.xw >> (c * VEC)) & ((1u << VEC) - 1u)) & vmask;
    L.sq = __builtin_amdgcn_sdot4((int)L.qw[c], 0x01010101, L.sq, false);
  }
}

// exact-path i side: t_i and the int8 rows (targets, and inputs for the
// kinetic search) as in k_score
template <class R, int NPL, int MODEL>
__device__ __forceinline__ void load_i_exact(const Fields& F, int i, R (&ti)[NPL], int (&yb)[NPL < 4 ? 1 : NPL / 4],
                                             int (&xb)[NPL < 4 ? 1 : NPL / 4], int lane) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int64_t row = (int64_t)i * F.Mp;
  const R* Tr = reinterpret_cast<const R*>(F.T) + row;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = smp<VEC>(c, lane);
    ld_vec<VEC>(Tr + o, ti + c * VEC);
    yb[c] = ld_bytes<VEC>((MODEL == REC_KINSYM ? F.ys : F.xs) + row + o);
    if constexpr (MODEL == REC_KINSYM) xb[c] = ld_bytes<VEC>(F.xs + row + o);
  }
}

// Screened scoring runs as two kernels.  k_kink settles every side whose
// kink test is decided by the fast sums and writes the zero gains; it keeps
// only the resident r_i row, sign words and the prefetched screen data in
// registers, so many waves fit per SIMD and many j rows are in flight.  The
// rest (a few percent of the pairs) go to a queue, and k_exact scores them
// with the full arithmetic.  Queue entry: pair index | QA (side i <- j, or
// the whole Ising pair) | QB (side j <- i of the kinetic search).
constexpr uint32_t QA = 1u << 30, QB = 1u << 31, QIDX = QA - 1;

template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_kink(Fields F, WTable W, int64_t P,
                                              const int32_t* __restrict__ I,
                                              const int32_t* __restrict__ J,
                                              const int32_t* __restrict__ Smap,
                                              const uint32_t* __restrict__ slot, int owned,
                                              double* __restrict__ gain_out,
                                              double* __restrict__ w_out,
                                              double* __restrict__ ovf, uint64_t cache_cap,
                                              int32_t* err, int ppw, int groups,
                                              uint32_t* __restrict__ queue, int64_t* qn,
                                              int64_t qcap, int64_t* work) {
  constexpr bool SYM = MODEL == REC_KINSYM;
  const int lane = rec_lane();
  // (uniform: the pair addresses derived from it stay scalar)
  const int64_t wave = rec_uni((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE));
  // byte -> its bits spread to the nibbles of a word (rec_spread8), one LDS
  // read instead of nine ALU operations per word of signs
  __shared__ uint32_t spread[256];
  for (int t = threadIdx.x; t < 256; t += blockDim.x) spread[t] = rec_spread8((uint32_t)t);
  __syncthreads();
  // a wave walks `groups` consecutive groups of ppw slots (owner mode: most
  // slots are cache hits, so one group holds few pairs; the i row and the
  // wave's set-up are shared by the groups)
  const int64_t wbeg = wave * ppw * groups;
  if (wbeg >= P) return;
  LaneR<R, NPL> L;
  constexpr int KD = NPL >= 32 ? 3 : 6;
  JScr<NPL, SYM> nx[KD];   // screen data of the next KD pairs, in flight
  int cur = -1;
  Work wk;
  int32_t n_items = 0, n_settled = 0;   // pairs (sides) tested and settled, 32-bit scalar counts
  for (int g = 0; g < groups; ++g) {
  uint32_t mine = 0;   // lane q: queue entry of the group's pair q (0: none)
  uint64_t settled = 0;   // bit q: pair q settled at the kink, its zeros stored after the group
  const int64_t p0 = wbeg + (int64_t)g * ppw;
  if (p0 >= P) break;
  int np = (int)(p0 + ppw < P ? ppw : P - p0);
  int li = -1, lj = -1;
  double lw = 0.0, lw2 = 0.0;
  if (lane < np) {
    uint32_t sw = slot ? slot[p0 + lane] : 0u;
    if (owned && !(sw & OWNER)) {
      li = SKIP;
    } else {
      li = I[p0 + lane];
      lj = J[p0 + lane];
      if (Smap) lj = Smap[lj];
    }
  }
  // the group's pairs checked once, one per lane: the loop below takes only
  // valid ones; an invalid pair gets NaN and the error bit here
  const bool lane_pair = lane < np && li != SKIP;
  const bool lane_ok = lane_pair && pair_ok(li, lj, F.N);
  uint64_t todo = __ballot(lane_ok);
  if (lane_pair && !lane_ok) {
    const int64_t p = p0 + lane;
    double* dst = gain_out + p;
    if (slot) {
      const uint64_t o = (uint64_t)(slot[p] & ~OWNER);
      dst = o >= cache_cap ? ovf + (o - cache_cap) : gain_out + o;
    }
    *dst = __builtin_nan("");
    if (w_out) w_out[p] = __builtin_nan("");
    atomicOr(err, 1);
  }
  if constexpr (!SYM) n_items += __builtin_popcountll(todo);
  uint64_t pf = todo;   // pairs whose screen data is not yet requested
  auto prefetch = [&](JScr<NPL, SYM>& dst) {
    const int qq = __ffsll((unsigned long long)pf) - 1;
    pf &= pf - 1;
    fetch_scr<NPL, SYM>(F, rec_lane_val(lj, qq), dst, lane);
  };
  // four pairs' screen data in flight ahead of the one being tested, issued
  // before the weight lookups (hash probes) so that the probes' latency
  // overlaps the rows' (and the first i row's)
#pragma unroll
  for (int d = 0; d < KD; ++d)
    if (pf) prefetch(nx[d]);
  if (todo && g == 0) {
    const int i0 = rec_lane_val(li, __ffsll((unsigned long long)todo) - 1);
    if (i0 >= 0 && i0 < F.N) { load_i_r<R, NPL, MODEL>(F, i0, L, lane); cur = i0; ++wk.iloads; }
  }
  if (lane_ok) {
    lw = lookup_w(W, li, lj, SYM);
    if constexpr (SYM) lw2 = lookup_w(W, lj, li, true);
  }
  // bit q: pair q's current weight(s) are zero (+-0)
  const uint64_t wz = __ballot(lw == 0.0);
  const uint64_t wz2 = SYM ? __ballot(lw2 == 0.0) : 0ull;
  // Pair t of the group uses slot t % KD of the ring, refilled with pair
  // t + KD's data once the pair is tested: no register moves between slots.
  while (todo) {
#pragma unroll
  for (int d = 0; d < KD; ++d) {
    if (!todo) break;
    const int q = __ffsll((unsigned long long)todo) - 1;
    todo &= todo - 1;
    const int64_t p = p0 + q;
    const int i = rec_lane_val(li, q), j = rec_lane_val(lj, q);
    const bool w0z = (wz >> q) & 1ull;
    const JScr<NPL, SYM>& rw = nx[d];
    if (i != cur) { load_i_r<R, NPL, MODEL>(F, i, L, lane); cur = i; ++wk.iloads; }
    // The kink test in two stages.  First from the 4-bit copies u of
    // 1 - y t (y - t = y u): with s = +-1 the product of two signs and
    // b = (s + 1) / 2 as nibbles, sum s u = 2 (sum of u where s = +1) - sum u,
    // in exact integers by 8-way nibble dot products (7.5 x the screened sum);
    // a side it leaves open takes the int8 test, then the exact path.
    constexpr int UW = LaneR<R, NPL>::UW;
    bool na, nb = false;
    if constexpr (MODEL == REC_ISING) {
      // Phi(0) = sum x_i x_j (u_i + u_j) (y = x)
      const uint32_t sx = ~(L.xw ^ rw.xw);
      uint32_t v = 0, uj = 0;
#pragma unroll
      for (int w = 0; w < UW; ++w) {
        const uint32_t b = spread[(sx >> (8 * w)) & 0xffu];
        v = __builtin_amdgcn_udot8(b, L.ui[w], v, false);
        v = __builtin_amdgcn_udot8(b, rw.uw[w], v, false);
        uj = __builtin_amdgcn_udot8(0x11111111u, rw.uw[w], uj, false);
      }
      na = !w0z || abs(rec_wave_sum_dpp(2 * (int)v - L.su - (int)uj)) > F.t42;
      if (na && w0z) {
        uint32_t qw[LaneR<R, NPL>::CH];
        fetch_q8<NPL>(F, j, qw, lane);
        // sum x_j q_i = 2 (sum of q_i where x_j = +1) - sum q_i, and sum x_i q_j
        // against x_i's +-1 bytes (|.| <= 127 M: exact, also the wave sums)
        int sa = 0, sb = 0;
#pragma unroll
        for (int c = 0; c < LaneR<R, NPL>::CH; ++c) {
          constexpr int VEC = LaneR<R, NPL>::VEC;
          sa = __builtin_amdgcn_sdot4((int)L.qw[c], (int)spread01((rw.xw >> (c * VEC)) & ((1u << VEC) - 1u)), sa, false);
          sb = __builtin_amdgcn_sdot4((int)qw[c], (int)L.pm[c], sb, false);
        }
        sa = 2 * sa - L.sq;
        na = (float)abs(rec_wave_sum_dpp(sa + sb)) * REC_Q8_INV > F.scr2;
        ++wk.tfetch;
      }

    } else {
      // i <- j: sum x_j y_i u_i;  j <- i: sum x_i y_j u_j
      const bool w0bz = (wz2 >> q) & 1ull;
      const uint32_t sa4 = ~(rw.xw ^ L.yw), sb4 = ~(L.xw ^ rw.yw);
      uint32_t va = 0, vb = 0, uj = 0;
#pragma unroll
      for (int w = 0; w < UW; ++w) {
        va = __builtin_amdgcn_udot8(spread[(sa4 >> (8 * w)) & 0xffu], L.ui[w], va, false);
        vb = __builtin_amdgcn_udot8(spread[(sb4 >> (8 * w)) & 0xffu], rw.uw[w], vb, false);
        uj = __builtin_amdgcn_udot8(0x11111111u, rw.uw[w], uj, false);
      }
      na = !w0z || abs(rec_wave_sum_dpp(2 * (int)va - L.su)) > F.t4;
      nb = !w0bz || abs(rec_wave_sum_dpp(2 * (int)vb - (int)uj)) > F.t4;
      if ((na && w0z) || (nb && w0bz)) {
        uint32_t qw[LaneR<R, NPL>::CH];
        fetch_q8<NPL>(F, j, qw, lane);
        int sa = 0, sb = 0;
#pragma unroll
        for (int c = 0; c < LaneR<R, NPL>::CH; ++c) {
          constexpr int VEC = LaneR<R, NPL>::VEC;
          sa = __builtin_amdgcn_sdot4((int)L.qw[c], (int)spread01((rw.xw >> (c * VEC)) & ((1u << VEC) - 1u)), sa, false);
          sb = __builtin_amdgcn_sdot4((int)qw[c], (int)L.pm[c], sb, false);
        }
        sa = 2 * sa - L.sq;
        if (na && w0z) na = (float)abs(rec_wave_sum_dpp(sa)) * REC_Q8_INV > F.scr;
        if (nb && w0bz) nb = (float)abs(rec_wave_sum_dpp(sb)) * REC_Q8_INV > F.scr;
        ++wk.tfetch;
      }
      n_items += 2;
      n_settled += (na ? 0 : 1) + (nb ? 0 : 1);
    }
    if (!na && !nb) {
      settled |= 1ull << q;
    } else if (lane == q) {
      mine = (uint32_t)p | (na ? QA : 0u) | (nb ? QB : 0u);
    }
    if (pf) prefetch(nx[d]);
  }
  }
  if constexpr (!SYM) n_settled += __builtin_popcountll(settled);
  // the settled pairs' zeros, lane q for pair q
  if ((settled >> lane) & 1ull) {
    const int64_t p = p0 + lane;
    double* dst = gain_out + p;
    if (slot) {
      const uint64_t o = (uint64_t)(slot[p] & ~OWNER);
      dst = o >= cache_cap ? ovf + (o - cache_cap) : gain_out + o;
    }
    *dst = 0.0;
    if (w_out) w_out[p] = 0.0;
  }
  // one atomic per wave and group for the queued pairs
  const int64_t pos = rec_append(qn, mine != 0u);
  if (pos >= 0) {
    if (pos < qcap) queue[pos] = mine;
    else atomicOr(err, 512);
  }
  }
  wk.pairs += n_items;
  wk.screened += n_settled;
  if (lane == 0 && work) {
    const int64_t M = F.M;
    const int64_t items = SYM ? wk.pairs / 2 : wk.pairs;
    const int64_t sb = (M + 7) / 8 * (SYM ? 2 : 1);   // sign words
    // per pair: indices and score, the j side's signs and 4-bit copies (plus
    // its int8 row when the 4-bit test left a side open); per i load: its
    // signs, 4-bit copies and int8 row
    wk.bytes = items * (16 + (slot ? 4 : 0) + sb + (M + 1) / 2) + wk.tfetch * M +
               wk.iloads * (sb + (M + 1) / 2 + M);
    wk.tfetch = 0;   // (int8 rows, not tanh rows: counted in the bytes)
    wk.flush(work, wave);
  }
}

// The queued pairs, in contiguous ranges per wave (consecutive entries
// usually share i, whose exact rows are then loaded once).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) void k_exact(Fields F, WTable W, double lambda,
                                               const int32_t* __restrict__ I,
                                               const int32_t* __restrict__ J,
                                               const int32_t* __restrict__ Smap,
                                               const uint32_t* __restrict__ slot,
                                               double* __restrict__ gain_out,
                                               double* __restrict__ w_out,
                                               double* __restrict__ ovf, uint64_t cache_cap,
                                               const uint32_t* __restrict__ queue,
                                               const int64_t* __restrict__ qn, int64_t qcap,
                                               int64_t* work) {
  constexpr bool SYM = MODEL == REC_KINSYM;
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int lane = rec_lane();
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / REC_WAVE);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE;
  int64_t n = *qn;
  if (n > qcap) n = qcap;
  const int64_t per = (n + nwaves - 1) / nwaves;
  const int64_t e0 = wave * per, e1 = e0 + per < n ? e0 + per : n;
  Work wk;
  R ti[NPL], wv[NPL];
  int yb[CH], xb[CH];
  int cur = -1;
  for (int64_t e = e0; e < e1; ++e) {
    const uint32_t ent = queue[e];
    const int64_t p = ent & QIDX;
    const bool na = (ent & QA) != 0, nb = (ent & QB) != 0;
    const int i = rec_uni(I[p]);
    int j = J[p];
    if (Smap) j = Smap[j];
    j = rec_uni(j);
    double* dst = gain_out + p;
    if (slot) {
      const uint64_t o = (uint64_t)(slot[p] & ~OWNER);
      dst = o >= cache_cap ? ovf + (o - cache_cap) : gain_out + o;
    }
    if (i != cur) { load_i_exact<R, NPL, MODEL>(F, i, ti, yb, xb, lane); cur = i; ++wk.iloads; }
    const uint32_t xw = rec_sign_word<NPL>(F.xq, j, lane);
    PairOut r;
    if constexpr (MODEL == REC_ISING) {
      const double w0 = rec_uni(lookup_w(W, i, j, false));
      ++wk.tfetch;
      R u[NPL];
      fetch_t<R, NPL>(F, j, wv, lane);
      float s = 0.f;
      R a = R(0), a2 = R(0);
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          const int qq = c * VEC + k;
          float xj = sgn_at(xw, qq);
          float xi = byte_at(yb[c], k);
          R uu = (R)xj * ti[qq];
          u[qq] = uu;
          a += uu;
          R v = (R)xi * wv[qq];
          wv[qq] = v;
          a2 += v;
          s += xj * xi;
        }
      double phi0 = rec_wave_sum_dpp(2.0 * (double)s - ((double)a + (double)a2));
      r = solve_ising<R, NPL, true>(u, wv, phi0, s, w0, lambda, F.M, F.Mp, wk);
    } else {
      const double w0 = rec_uni(lookup_w(W, i, j, true));
      const double w0b = rec_uni(lookup_w(W, j, i, true));
      PairOut ra, rb;
      ra.gain = 0.0; ra.w = 0.0; ra.w0 = w0;
      rb.gain = 0.0; rb.w = 0.0; rb.w0 = w0b;
      if (na) {
        float s1 = 0.f;
        R a = R(0);
#pragma unroll
        for (int c = 0; c < CH; ++c)
#pragma unroll
          for (int k = 0; k < VEC; ++k) {
            const int qq = c * VEC + k;
            float xj = sgn_at(xw, qq);
            R uu = (R)xj * ti[qq];
            wv[qq] = uu;
            a += uu;
            s1 += xj * byte_at(yb[c], k);
          }
        double pa = rec_wave_sum_dpp((double)s1 - (double)a);
        ra = solve_ising<R, NPL, false>(wv, wv, pa, s1, w0, lambda, F.M, F.Mp, wk);
      }
      if (nb) {
        ++wk.tfetch;
        const uint32_t yw = rec_sign_word<NPL>(F.yq, j, lane);
        fetch_t<R, NPL>(F, j, wv, lane);
        float s2 = 0.f;
        R b = R(0);
#pragma unroll
        for (int c = 0; c < CH; ++c)
#pragma unroll
          for (int k = 0; k < VEC; ++k) {
            const int qq = c * VEC + k;
            float xi = byte_at(xb[c], k);
            R v = (R)xi * wv[qq];
            wv[qq] = v;
            b += v;
            s2 += xi * sgn_at(yw, qq);
          }
        double pb = rec_wave_sum_dpp((double)s2 - (double)b);
        rb = solve_ising<R, NPL, false>(wv, wv, pb, s2, w0b, lambda, F.M, F.Mp, wk);
      }
      r = rb.gain > ra.gain ? rb : ra;
    }
    double g = r.gain;
    if constexpr (sizeof(R) == 4) g = (double)(float)g;   // FP32 scores
    if (lane == 0) {
      *dst = g;
      if (w_out) w_out[p] = r.w;
    }
  }
  if (lane == 0 && work) {
    const int64_t M = F.M, rs = sizeof(R);
    wk.bytes = wk.tfetch * rs * M + wk.iloads * (rs * M + M * (SYM ? 2 : 1)) + (e1 > e0 ? (e1 - e0) * 24 : 0);
    wk.flush(work, wave);
  }
}

// Solve pair p of the rank-ordered list and apply its update (one wave).
template <class R, int NPL, int MODEL>
__device__ __forceinline__ void update_pair(const Fields& F, const WTable& W, double lambda, int64_t p,
                                            const int32_t* __restrict__ I,
                                            const int32_t* __restrict__ J,
                                            const int64_t* __restrict__ wslot, uint8_t* done,
                                            double* dw) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int lane = rec_lane();
  const int i = I[p], j = J[p];
  const int64_t ws = wslot[p];
  Lane<R, NPL> L;
  load_i<R, NPL, MODEL>(F, i, L, lane);
  JRaw<R, NPL, MODEL> rw;
  fetch_j<R, NPL, MODEL>(F, j, rw, lane);
  float s_lane;
  double phi_l = form_j<R, NPL, MODEL>(rw, L, &s_lane);
  double phi0 = MODEL == REC_GAUSS ? 0.0 : rec_wave_sum_dpp(phi_l);
  const double w0 = rec_uni(ws >= 0 ? W.vals[ws] : 0.0);
  Work wk;
  PairOut r = solve<R, NPL, MODEL>(F, L, phi0, s_lane, i, j, w0, lambda, wk);
  double d = r.w - w0;
  if (d != 0.0) {
    // rows of H (and T): h_i += d x_j, h_j += d x_i [App. A, O(1) field bookkeeping]
    R* H = reinterpret_cast<R*>(F.H);
    R* T = reinterpret_cast<R*>(F.T);
    for (int side = 0; side < (MODEL == REC_KINETIC ? 1 : 2); ++side) {
      int row = side == 0 ? i : j, other = side == 0 ? j : i;
      double scale = d;
      if constexpr (MODEL == REC_GAUSS) scale = d * F.theta[row] * F.theta[row];
      constexpr int UW = rec_u4_words(NPL);
      uint32_t uw[UW];
#pragma unroll
      for (int w = 0; w < UW; ++w) uw[w] = 0u;
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        int64_t o = smp<VEC>(c, lane);
        float xv[VEC];
        R hv[VEC];
        if constexpr (MODEL == REC_GAUSS) {
          // the wave holds both rows already: r_i (= h_i) and x_i as the i
          // side, x_j and r_j as the j side; no other wave writes them now
#pragma unroll
          for (int k = 0; k < VEC; ++k) {
            const int q = c * VEC + k;
            xv[k] = side == 0 ? (float)L.u[q] : (float)L.xi[q];
            hv[k] = side == 0 ? L.ti[q] : L.v[q];
          }
        } else {
          ld_x<VEC>(F.xs + (int64_t)other * F.Mp + o, xv);
#pragma unroll
          for (int k = 0; k < VEC; ++k) hv[k] = H[(int64_t)row * F.Mp + o + k];
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          int64_t idx = (int64_t)row * F.Mp + o + k;
          R h = hv[k] + (R)(scale * (double)xv[k]);
          if (o + k < F.M) {
            H[idx] = h;
            if constexpr (MODEL != REC_GAUSS) {
              R t = tanh_(h);
              T[idx] = t;
              const int8_t* Y = MODEL == REC_KINETIC ? F.ys : F.xs;
              const R yv = (R)Y[idx];
              F.rq[idx] = rec_q8((float)(yv - t));
              const int n = c * VEC + k;
              uw[n >> 3] |= rec_u4((float)(R(1) - yv * t)) << (4 * (n & 7));
            }
          }
        }
      }
      if constexpr (MODEL != REC_GAUSS) {
#pragma unroll
        for (int w = 0; w < UW; ++w) F.u4[((int64_t)row * UW + w) * REC_WAVE + lane] = uw[w];
      }
    }
    if (lane == 0 && ws >= 0) W.vals[ws] = r.w;
  }
  if (lane == 0) {
    dw[p] = fabs(d);
    if (done) done[p] = 1;
  }
}

// One round of node-disjoint updates over the list ready[0..*nready) of pairs
// that are the earliest pending pair of each of their rows; such pairs touch
// disjoint rows, so the round equals the sequential rank order. The grid is
// sized for the device, not the list: each wave takes list entries in a
// grid-stride loop, so every resident wave solves a ready pair (each pair is a
// serial chain of loads and Newton steps: five waves per SIMD hide more of it
// than four for rows of up to 8 samples a lane; at 16 and more, five waves'
// 102 VGPRs spill (32 in FP32) and four waves without spills are faster, C4s
// updates 1.4-2.9 ms per sweep against 1.8-3.3).  W entries
// are reached through the slots reserved for the list before the rounds
// (wslot[p], no probing on the serial path of a pair); a pair's entry is
// written only by that pair, so its value is current when the pair runs.
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NPL >= 16 ? 4 : 5))) void k_update(Fields F, WTable W, double lambda,
                                                const int32_t* __restrict__ I,
                                                const int32_t* __restrict__ J,
                                                const int32_t* __restrict__ ready,
                                                const int64_t* __restrict__ nready,
                                                const int64_t* __restrict__ wslot, uint8_t* done,
                                                double* dw, int32_t* depth, int32_t round) {
  const int64_t n = *nready;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / REC_WAVE);
  for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE; q < n; q += nw) {
    const int32_t p = ready[q];
    update_pair<R, NPL, MODEL>(F, W, lambda, p, I, J, wslot, done, dw);
    if (rec_lane() == 0) depth[p] = round;
  }
}

// The last pairs of the node-disjoint schedule as a dataflow over the whole
// grid.  Once the rounds ready few pairs each (the runs of updates on hub
// rows), a round costs its three launches, not its work; here the pairs not
// yet done run without rounds.  Each wave takes the next rank from a ticket
// counter, skips it if the rounds did it, waits until the pair's
// predecessors on both rows are done, applies the update and publishes its
// done flag (2) after a release fence at device scope.  A predecessor done by
// the rounds (flag 1) is visible at the launch; one done in this launch
// (flag 2) is read after an acquire fence at device scope (the writer may sit
// on another XCD, behind another L2).  The order of the updates on every row
// is the rank order, so the results are those of the rounds, bit for bit.
//
// Progress: tickets are taken in rank order and a wave takes a ticket only
// while it runs, so the smallest taken and unfinished pair has all its
// predecessors (smaller ranks, all taken) finished and its wave running; it
// finishes, and by induction every pair does, whatever the residency of the
// grid.  The wait is bounded all the same: after spin_limit polls the wave
// raises an abort flag that every waiting wave reads, all waves leave, and the
// host reports the error (bit 1024).
//
// depth[p] = 1 + the larger depth of the predecessors, the round the pair
// would have run in; the largest goes to *rounds.
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NPL >= 16 ? 4 : 5))) void k_update_flow(
    Fields F, WTable W, double lambda, const int32_t* __restrict__ I, const int32_t* __restrict__ J, int64_t m,
    const int32_t* __restrict__ pred, const int64_t* __restrict__ wslot, uint8_t* done, double* dw,
    int32_t* depth, unsigned long long* ticket, unsigned long long* rounds, int64_t* abort_flag, int32_t* err,
    int64_t spin_limit) {
  const int lane = rec_lane();
  for (;;) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(ticket, 1ull);
    const int64_t p = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(t >> 32)) << 32) |
                                (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)t));
    if (p >= m) break;
    if (done[p] != 0) continue;   // done by the rounds (only this wave can run p here)
    const int32_t a = pred[2 * p], b = pred[2 * p + 1];
    int ok = 1, fresh = 0;
    if (lane == 0) {
      // poll only the flags not yet seen set; the abort flag every 32 polls;
      // a long wait polls less often (most waiting wavefronts sit far down a
      // chain, and their polls share the memory path with the chain's head)
      int fa = a < 0 ? 1 : 0, fb = b < 0 ? 1 : 0;
      for (int64_t polls = 0;; ++polls) {
        if (fa == 0) fa = __hip_atomic_load(done + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fb == 0) fb = __hip_atomic_load(done + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fa != 0 && fb != 0) {
          fresh = fa == 2 || fb == 2;
          break;
        }
        if (polls >= spin_limit ||
            ((polls & 31) == 31 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
          ok = 0;
          break;
        }
        if (polls < 64) __builtin_amdgcn_s_sleep(1);
        else __builtin_amdgcn_s_sleep(16);
      }
    }
    if (!__builtin_amdgcn_readfirstlane(ok)) {
      if (lane == 0) {
        __hip_atomic_store(abort_flag, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicOr(err, 1024);
      }
      break;
    }
    if (__builtin_amdgcn_readfirstlane(fresh)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // the predecessors' depths are read here, beside the pair's row loads,
    // not on the path from the update to the release
    int32_t d = 0;
    if (lane == 0) d = 1 + max(a < 0 ? 0 : depth[a], b < 0 ? 0 : depth[b]);
    update_pair<R, NPL, MODEL>(F, W, lambda, p, I, J, wslot, nullptr, dw);
    if (lane == 0) {
      depth[p] = d;
      atomicMax(rounds, (unsigned long long)d);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(done + p, (uint8_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One coordinate of a CD sweep [Alg. 1] (one wave): W_ij <- its argmax at the
// current state, with the arithmetic of update_pair, but the coupling found
// or created in the W table on the spot (a CD sweep visits every pair, so no
// slots are reserved beforehand; only changed couplings are written).
template <class R, int NPL, int MODEL>
__device__ __forceinline__ void cd_pair(const Fields& F, const WTable& W, double lambda, int i, int j,
                                        double* acc, int64_t* changes, int32_t* err) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  constexpr bool DIR = MODEL == REC_KINETIC;
  const int lane = rec_lane();
  Lane<R, NPL> L;
  load_i<R, NPL, MODEL>(F, i, L, lane);
  JRaw<R, NPL, MODEL> rw;
  fetch_j<R, NPL, MODEL>(F, j, rw, lane);
  float s_lane;
  double phi_l = form_j<R, NPL, MODEL>(rw, L, &s_lane);
  double phi0 = MODEL == REC_GAUSS ? 0.0 : rec_wave_sum_dpp(phi_l);
  const double w0 = rec_uni(lookup_w(W, i, j, DIR));
  Work wk;
  PairOut r = solve<R, NPL, MODEL>(F, L, phi0, s_lane, i, j, w0, lambda, wk);
  const double d = r.w - w0;
  if (d == 0.0) return;
  R* H = reinterpret_cast<R*>(F.H);
  R* T = reinterpret_cast<R*>(F.T);
  for (int side = 0; side < (DIR ? 1 : 2); ++side) {
    const int row = side == 0 ? i : j, other = side == 0 ? j : i;
    double scale = d;
    if constexpr (MODEL == REC_GAUSS) scale = d * F.theta[row] * F.theta[row];
    constexpr int UW = rec_u4_words(NPL);
    uint32_t uw[UW];
#pragma unroll
    for (int w = 0; w < UW; ++w) uw[w] = 0u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t o = smp<VEC>(c, lane);
      float xv[VEC];
      if constexpr (MODEL == REC_GAUSS) ld_f<VEC>(F.xf + (int64_t)other * F.Mp + o, xv);
      else ld_x<VEC>(F.xs + (int64_t)other * F.Mp + o, xv);
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const int64_t idx = (int64_t)row * F.Mp + o + k;
        const R h = H[idx] + (R)(scale * (double)xv[k]);
        if (o + k < F.M) {
          H[idx] = h;
          if constexpr (MODEL != REC_GAUSS) {
            const R t = tanh_(h);
            T[idx] = t;
            const int8_t* Y = MODEL == REC_KINETIC ? F.ys : F.xs;
            const R yv = (R)Y[idx];
            F.rq[idx] = rec_q8((float)(yv - t));
            const int n = c * VEC + k;
            uw[n >> 3] |= rec_u4((float)(R(1) - yv * t)) << (4 * (n & 7));
          }
        }
      }
    }
    if constexpr (MODEL != REC_GAUSS) {
#pragma unroll
      for (int w = 0; w < UW; ++w) F.u4[((int64_t)row * UW + w) * REC_WAVE + lane] = uw[w];
    }
  }
  if (lane == 0) {
    bool ins;
    const uint64_t key = rec_pair_key(i, j, DIR);
    const int64_t slot = rec_hash_insert(W.keys, W.mask, key, REC_MAX_PROBE, &ins);
    if (slot < 0) {
      atomicOr(err, 2);
    } else {
      rec_wbloom_set(W, key);
      W.vals[slot] = r.w;
    }
    *acc += fabs(d);
    atomicAdd((unsigned long long*)changes, 1ull);
  }
}

// Round r of a round-robin CD sweep over n = N rounded up to even nodes
// (node n - 1 a phantom when N is odd): pair k pairs r with n - 1 (k = 0) or
// (r + k) mod (n - 1) with (r - k) mod (n - 1).  The round's pairs share no
// node, so they run in parallel exactly as in sequence.  acc[k] collects pair
// k's |dW| over the rounds (one wave per k and round, so its sum is fixed).
// Symmetric models update (min, max); the kinetic model both ordered
// couplings, (a <- b) then (b <- a).
template <class R, int NPL, int MODEL>
__global__ __launch_bounds__(256) void k_cd_round(Fields F, WTable W, double lambda, int64_t r,
                                                  int64_t n, double* acc, int64_t* changes,
                                                  int32_t* err) {
  const int64_t half = n / 2;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / REC_WAVE);
  for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / REC_WAVE; k < half; k += nw) {
    int64_t a, b;
    if (k == 0) { a = r; b = n - 1; }
    else { a = (r + k) % (n - 1); b = (r - k + (n - 1)) % (n - 1); }
    if (a >= F.N || b >= F.N) continue;
    if constexpr (MODEL == REC_KINETIC) {
      cd_pair<R, NPL, MODEL>(F, W, lambda, (int)a, (int)b, acc + k, changes, err);
      cd_pair<R, NPL, MODEL>(F, W, lambda, (int)b, (int)a, acc + k, changes, err);
    } else {
      cd_pair<R, NPL, MODEL>(F, W, lambda, (int)(a < b ? a : b), (int)(a < b ? b : a), acc + k, changes, err);
    }
  }
}

// The chain of updates of one target row i of a directed model, in rank
// order (one wave): the row's fields h_i stay in the lanes' registers from
// the chain's first pair to its last, and h_i, t_i = tanh h_i and the int8
// residuals y_i - t_i are written once at the end; every pair sees the
// fields left by the one before it, as in the sequential order.  Each step
// has the arithmetic of update_pair, so the results are the same bit for
// bit.  The current weight is read by lane 0, the lane that writes it, so a
// pair listed twice in one chain sees its first update.
template <class R, int NPL>
__device__ __forceinline__ void update_chain(const Fields& F, const WTable& W, double lambda,
                                             const int32_t* __restrict__ cpair, int64_t e0, int64_t n,
                                             const int32_t* __restrict__ I,
                                             const int32_t* __restrict__ J,
                                             const int64_t* __restrict__ wslot, uint8_t* done,
                                             double* dw) {
  constexpr int VEC = NPL < 4 ? NPL : 4, CH = NPL / VEC;
  const int lane = rec_lane();
  const int i = I[cpair[e0]];
  const int64_t row = (int64_t)i * F.Mp;
  R* H = reinterpret_cast<R*>(F.H);
  R* T = reinterpret_cast<R*>(F.T);
  R h[NPL], u[NPL];
  int yb[CH];   // targets y_i, VEC bytes per chunk
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int64_t o = smp<VEC>(c, lane);
    ld_vec<VEC>(H + row + o, h + c * VEC);
    yb[c] = ld_bytes<VEC>(F.ys + row + o);
  }
  bool changed = false;
  for (int64_t e = e0; e < e0 + n; ++e) {
    const int32_t p = cpair[e];
    const int j = J[p];
    const int64_t ws = wslot[p];
    // sample terms u = x_j t_i, their sum and the lane's part of S = sum y_i x_j;
    // t_i from T until the chain first changes the row, then tanh h_i, the
    // value the row's store would have held (padding: h = t = 0)
    float s_lane = 0.f;
    R a = R(0);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t o = smp<VEC>(c, lane);
      const int xw = ld_bytes<VEC>(F.xs + (int64_t)j * F.Mp + o);
      R tv[VEC];
      if (changed) {
#pragma unroll
        for (int k = 0; k < VEC; ++k) tv[k] = tanh_(h[c * VEC + k]);
      } else {
        ld_vec<VEC>(T + row + o, tv);
      }
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const float x = byte_at(xw, k);
        const R uq = (R)x * tv[k];
        u[c * VEC + k] = uq;
        a += uq;
        s_lane += x * byte_at(yb[c], k);
      }
    }
    const double phi0 = rec_wave_sum_dpp((double)s_lane - (double)a);
    double wl = 0.0;
    if (lane == 0 && ws >= 0)
      wl = __builtin_bit_cast(double, __atomic_load_n(reinterpret_cast<const uint64_t*>(W.vals + ws), __ATOMIC_RELAXED));
    const double w0 = rec_lane_val(wl, 0);
    Work wk;
    const PairOut r = solve_ising<R, NPL, false>(u, u, phi0, s_lane, w0, lambda, F.M, F.Mp, wk);
    const double d = r.w - w0;
    if (d != 0.0) {
      // h_i += d x_j [App. A]; x_j read again rather than held across the solve
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int64_t o = smp<VEC>(c, lane);
        const int xw = ld_bytes<VEC>(F.xs + (int64_t)j * F.Mp + o);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          const R hn = h[c * VEC + k] + (R)(d * (double)byte_at(xw, k));
          if (o + k < F.M) h[c * VEC + k] = hn;
        }
      }
      changed = true;
      if (lane == 0 && ws >= 0) W.vals[ws] = r.w;
    }
    if (lane == 0) {
      dw[p] = fabs(d);
      done[p] = 1;
    }
  }
  if (changed) {
    constexpr int UW = rec_u4_words(NPL);
    uint32_t uw[UW];
#pragma unroll
    for (int w = 0; w < UW; ++w) uw[w] = 0u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t o = smp<VEC>(c, lane);
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const int q = c * VEC + k;
        if (o + k < F.M) {
          const R t = tanh_(h[q]);
          H[row + o + k] = h[q];
          T[row + o + k] = t;
          const R yv = (R)byte_at(yb[c], k);
          F.rq[row + o + k] = rec_q8((float)(yv - t));
          uw[q >> 3] |= rec_u4((float)(R(1) - yv * t)) << (4 * (q & 7));
        }
      }
    }
    const int64_t r = row / F.Mp;
#pragma unroll
    for (int w = 0; w < UW; ++w) F.u4[(r * UW + w) * REC_WAVE + lane] = uw[w];
  }
}

// Directed couplings change only their target row's fields, so the
// rank-ordered updates split into independent chains, one per target row,
// each sequential in rank order [Alg. 2].  One wave runs one whole chain,
// taking chains from a queue ordered longest first (chain q: sorted entry
// key[q], low word = first position in cpair, length len[q]; keys with high
// byte 0xFF mark positions that start no chain and sort last).
template <class R, int NPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_update_chains(
    Fields F, WTable W, double lambda, const int32_t* __restrict__ I, const int32_t* __restrict__ J,
    const uint64_t* __restrict__ key, const uint32_t* __restrict__ len,
    const int32_t* __restrict__ cpair, int64_t n, unsigned long long* head,
    const int64_t* __restrict__ wslot, uint8_t* done, double* dw) {
  const int lane = rec_lane();
  while (true) {
    int q = 0;
    if (lane == 0) {
      const unsigned long long hd = atomicAdd(head, 1ull);
      q = hd < (unsigned long long)n ? (int)hd : -1;
    }
    q = rec_lane_val(q, 0);
    if (q < 0) break;
    const uint64_t k = key[q];
    if ((k >> 32) == 0xFF) break;
    update_chain<R, NPL>(F, W, lambda, cpair, (int64_t)(uint32_t)k, (int64_t)len[q], I, J, wslot, done, dw);
  }
}

// One 64-bit counter to zero (a kernel node, not a memset node, in a captured graph).
__global__ void k_zero_i64(int64_t* p) { *p = 0; }

template <class R, int MODEL>
rec_status launch_score_m(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                          const int32_t* Smap, const uint32_t* slot, int owned, double* gain_out,
                          double* w_out, const Cache* C, const ScoreScratch& ss) {
  // an empty W (right after a clear: W = 0) is passed without keys, and the
  // kernels take w = 0 without probing it
  WTable Wl = ctx->W;
  if (!ctx->w_any) Wl.keys = nullptr;
  // pairs per wave: owner mode reads 64 candidates, of which only the owned
  // (new) pairs are scored: most candidates after the first iteration are cache hits
  const int ppw = owned ? 64 : 32;
  int64_t waves = (P + ppw - 1) / ppw;
  int64_t blocks = (waves * REC_WAVE + 255) / 256;
  double* ovf = C ? C->ovf : nullptr;
  uint64_t cap = C ? (C->mask + 1) : 0;
  int64_t* ev = ss.work;
  if constexpr (MODEL == REC_ISING || MODEL == REC_KINSYM) {
    // settled sides in k_kink, the queue of the rest in k_exact (chunks of at
    // most the queue's capacity)
    int64_t* qn = ss.qn;
    const int64_t qcap = ss.qcap;
    const int64_t exact_blocks = 2048;
    for (int64_t c0 = 0; c0 < P; c0 += qcap) {
      const int64_t pc = P - c0 < qcap ? P - c0 : qcap;
      const int groups = owned ? 4 : 1;
      const int64_t span = (int64_t)ppw * groups;
      const int64_t cw = (pc + span - 1) / span, cb = (cw * REC_WAVE + 255) / 256;
      const int32_t* Ic = I + c0;
      const int32_t* Jc = J + c0;
      const uint32_t* sc = slot ? slot + c0 : nullptr;
      double* gc = slot ? gain_out : gain_out + c0;
      double* wc = w_out ? w_out + c0 : nullptr;
      if (ss.fill) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, ctx->stream, qn);
      else REC_HIP(hipMemsetAsync(qn, 0, sizeof(int64_t), ctx->stream));
#define REC_SC(NPL)                                                                              \
      hipLaunchKernelGGL((k_kink<R, NPL, MODEL>), dim3(cb), dim3(256), 0, ctx->stream, ctx->F,   \
                         Wl, pc, Ic, Jc, Smap, sc, owned, gc, wc, ovf, cap, ss.err,          \
                         ppw, groups, ss.queue, qn, qcap, ev);                                   \
      hipLaunchKernelGGL((k_exact<R, NPL, MODEL>), dim3(exact_blocks), dim3(256), 0, ctx->stream, \
                         ctx->F, Wl, ctx->cfg.lambda, Ic, Jc, Smap, sc, gc, wc, ovf, cap,        \
                         ss.queue, qn, qcap, ev)
      switch (ctx->F.npl) {
        case 1: REC_SC(1); break;
        case 2: REC_SC(2); break;
        case 4: REC_SC(4); break;
        case 8: REC_SC(8); break;
        case 16: REC_SC(16); break;
        case 32: REC_SC(32); break;
        default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
      }
#undef REC_SC
    }
    REC_HIP(hipGetLastError());
    return REC_OK;
  }
#define REC_SC(NPL)                                                                              \
  hipLaunchKernelGGL((k_score<R, NPL, MODEL>), dim3(blocks), dim3(256), 0, ctx->stream,          \
                     ctx->F, Wl, ctx->cfg.lambda, P, I, J, Smap, slot, owned, gain_out,          \
                     w_out, ovf, cap, ss.err, ppw, ev)
  switch (ctx->F.npl) {
    case 1: REC_SC(1); break;
    case 2: REC_SC(2); break;
    case 4: REC_SC(4); break;
    case 8: REC_SC(8); break;
    case 16: REC_SC(16); break;
    case 32: REC_SC(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_SC
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R, int MODEL>
rec_status launch_update_m(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                           const int32_t* ready, const int64_t* nready, uint8_t* done, double* dw,
                           int32_t* depth, int32_t round) {
  // enough 4-wave blocks to fill every CU a few times over, never more than the pairs
  const int64_t blocks = std::min<int64_t>((m + 3) / 4, 256 * 8);
#define REC_UP(NPL)                                                                              \
  hipLaunchKernelGGL((k_update<R, NPL, MODEL>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, \
                     ctx->F, ctx->W, ctx->cfg.lambda, I, J, ready, nready, ctx->best_slot, done, dw, depth, round)
  switch (ctx->F.npl) {
    case 1: REC_UP(1); break;
    case 2: REC_UP(2); break;
    case 4: REC_UP(4); break;
    case 8: REC_UP(8); break;
    case 16: REC_UP(16); break;
    case 32: REC_UP(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_UP
  REC_HIP(hipGetLastError());
  return REC_OK;
}

// 64 blocks of 4 waves (8 per XCD), never more waves than pairs: the launch
// starts once the rounds ready fewer than a few hundred pairs each, so more
// wavefronts would mostly wait, and their polls slow the loads of the pairs
// that run (C3 updates per sweep: 1280 blocks 30-38 ms, 256 blocks 18-24 ms,
// 64 or 32 blocks 10-17 ms, 8 blocks 14-19 ms).
template <class R, int MODEL>
rec_status launch_update_flow_m(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J, const int32_t* pred,
                                uint8_t* done, double* dw, int32_t* depth, int64_t* ticket, int64_t* rounds,
                                int64_t* abort_flag, int64_t spin_limit) {
  const int64_t blocks = std::min<int64_t>((m + 3) / 4, 64);
#define REC_UP(NPL)                                                                                          \
  hipLaunchKernelGGL((k_update_flow<R, NPL, MODEL>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream,       \
                     ctx->F, ctx->W, ctx->cfg.lambda, I, J, m, pred, ctx->best_slot, done, dw, depth,         \
                     reinterpret_cast<unsigned long long*>(ticket), reinterpret_cast<unsigned long long*>(rounds), \
                     abort_flag, ctx->err_flag, spin_limit)
  switch (ctx->F.npl) {
    case 1: REC_UP(1); break;
    case 2: REC_UP(2); break;
    case 4: REC_UP(4); break;
    case 8: REC_UP(8); break;
    case 16: REC_UP(16); break;
    case 32: REC_UP(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_UP
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R>
rec_status launch_update_flow_r(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J, const int32_t* pred,
                                uint8_t* done, double* dw, int32_t* depth, int64_t* ticket, int64_t* rounds,
                                int64_t* abort_flag, int64_t spin_limit) {
  switch (ctx->cfg.model) {
    case REC_ISING:
      return launch_update_flow_m<R, REC_ISING>(ctx, m, I, J, pred, done, dw, depth, ticket, rounds, abort_flag,
                                                spin_limit);
    case REC_GAUSS:
      return launch_update_flow_m<R, REC_GAUSS>(ctx, m, I, J, pred, done, dw, depth, ticket, rounds, abort_flag,
                                                spin_limit);
    case REC_KINETIC:
      return launch_update_flow_m<R, REC_KINETIC>(ctx, m, I, J, pred, done, dw, depth, ticket, rounds,
                                                  abort_flag, spin_limit);
  }
  return REC_E_INVAL;
}

template <class R, int MODEL>
rec_status launch_grad_m(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                         const int32_t* Smap, const uint32_t* slot, int owned, double* g,
                         const Cache* C) {
  WTable Wl = ctx->W;   // without keys while W is empty, as for the scores
  if (!ctx->w_any) Wl.keys = nullptr;
  const int ppw = owned ? 64 : 8;
  const int64_t waves = (P + ppw - 1) / ppw;
  const int64_t blocks = (waves * REC_WAVE + 255) / 256;
#define REC_GR(NPL)                                                                                    \
  hipLaunchKernelGGL((k_grad<R, NPL, MODEL>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, ctx->F, \
                     Wl, ctx->cfg.lambda, P, I, J, Smap, slot, owned, g, C ? C->ovf : nullptr,          \
                     C ? (C->mask + 1) : (uint64_t)0, ctx->err_flag, ppw, ctx->work)
  switch (ctx->F.npl) {
    case 1: REC_GR(1); break;
    case 2: REC_GR(2); break;
    case 4: REC_GR(4); break;
    case 8: REC_GR(8); break;
    case 16: REC_GR(16); break;
    case 32: REC_GR(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_GR
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R>
rec_status launch_score_r(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                          const int32_t* Smap, const uint32_t* slot, int owned, double* g,
                          double* w, const Cache* C, const ScoreScratch& ss) {
  if (ctx->grad_dist) {   // search under the gradient distance (no w*)
    switch (ctx->cfg.model) {
      case REC_ISING: return launch_grad_m<R, REC_ISING>(ctx, P, I, J, Smap, slot, owned, g, C);
      case REC_GAUSS: return launch_grad_m<R, REC_GAUSS>(ctx, P, I, J, Smap, slot, owned, g, C);
      case REC_KINETIC:
        if (ctx->sym_search) return launch_grad_m<R, REC_KINSYM>(ctx, P, I, J, Smap, slot, owned, g, C);
        return launch_grad_m<R, REC_KINETIC>(ctx, P, I, J, Smap, slot, owned, g, C);
    }
    return REC_E_INVAL;
  }
  switch (ctx->cfg.model) {
    case REC_ISING: return launch_score_m<R, REC_ISING>(ctx, P, I, J, Smap, slot, owned, g, w, C, ss);
    case REC_GAUSS: return launch_score_m<R, REC_GAUSS>(ctx, P, I, J, Smap, slot, owned, g, w, C, ss);
    case REC_KINETIC:
      if (ctx->sym_search) return launch_score_m<R, REC_KINSYM>(ctx, P, I, J, Smap, slot, owned, g, w, C, ss);
      return launch_score_m<R, REC_KINETIC>(ctx, P, I, J, Smap, slot, owned, g, w, C, ss);
  }
  return REC_E_INVAL;
}

template <class R>
rec_status launch_chains_r(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                           const uint64_t* key, const uint32_t* len, const int32_t* cpair,
                           int64_t n, int64_t* head, uint8_t* done, double* dw) {
  if (ctx->cfg.model != REC_KINETIC) { ctx->err = "update chains are for directed couplings"; return REC_E_INVAL; }
  const int64_t blocks = std::min<int64_t>((m + 3) / 4, 256 * 8);
  unsigned long long* hd = reinterpret_cast<unsigned long long*>(head);
#define REC_UC(NPL)                                                                              \
  hipLaunchKernelGGL((k_update_chains<R, NPL>), dim3((unsigned)blocks), dim3(256), 0, \
                     ctx->stream, ctx->F, ctx->W, ctx->cfg.lambda, I, J, key, len, cpair, n, hd, \
                     ctx->best_slot, done, dw)
  switch (ctx->F.npl) {
    case 1: REC_UC(1); break;
    case 2: REC_UC(2); break;
    case 4: REC_UC(4); break;
    case 8: REC_UC(8); break;
    case 16: REC_UC(16); break;
    case 32: REC_UC(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_UC
  REC_HIP(hipGetLastError());
  return REC_OK;
}

template <class R>
rec_status launch_update_r(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                           const int32_t* ready, const int64_t* nready, uint8_t* done, double* dw,
                           int32_t* depth, int32_t round) {
  switch (ctx->cfg.model) {
    case REC_ISING: return launch_update_m<R, REC_ISING>(ctx, m, I, J, ready, nready, done, dw, depth, round);
    case REC_GAUSS: return launch_update_m<R, REC_GAUSS>(ctx, m, I, J, ready, nready, done, dw, depth, round);
    case REC_KINETIC: return launch_update_m<R, REC_KINETIC>(ctx, m, I, J, ready, nready, done, dw, depth, round);
  }
  return REC_E_INVAL;
}

}  // namespace

rec_status rec_timing_resolve(rec_ctx* ctx) {
  for (size_t k = 0; k < ctx->ev_used; ++k) {
    REC_HIP(hipEventSynchronize(ctx->ev[k].second));
    float ms = 0.f;
    REC_HIP(hipEventElapsedTime(&ms, ctx->ev[k].first, ctx->ev[k].second));
    ctx->score_ms += ms;
  }
  ctx->ev_used = 0;
  return REC_OK;
}

namespace {
rec_status launch_score_any(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                            const int32_t* Smap, const uint32_t* slot, int owned,
                            double* gain_out, double* w_out, const Cache* cache);
}

rec_status rec_launch_score(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                            const uint32_t* slot, double* gain_out, double* w_out,
                            const Cache* cache) {
  return launch_score_any(ctx, P, I, J, nullptr, slot, 0, gain_out, w_out, cache);
}

rec_status rec_launch_score_owned(rec_ctx* ctx, int64_t P, const int32_t* gi, const int32_t* v,
                                  const int32_t* S, const uint32_t* slot, const Cache* cache) {
  return launch_score_any(ctx, P, gi, v, S, slot, 1, cache->vals, nullptr, cache);
}

rec_status rec_launch_score_with(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                                 double* gain_out, double* w_out, const ScoreScratch& ss) {
  if (P <= 0) return REC_OK;
  if (ctx->grad_dist) return REC_E_INVAL;
  return ctx->fp32 ? launch_score_r<float>(ctx, P, I, J, nullptr, nullptr, 0, gain_out, w_out, nullptr, ss)
                   : launch_score_r<double>(ctx, P, I, J, nullptr, nullptr, 0, gain_out, w_out, nullptr, ss);
}

namespace {
rec_status launch_score_any(rec_ctx* ctx, int64_t P, const int32_t* I, const int32_t* J,
                            const int32_t* Smap, const uint32_t* slot, int owned,
                            double* gain_out, double* w_out, const Cache* cache) {
  if (P <= 0) return REC_OK;
  if (ctx->timing) {
    if (ctx->ev_used == 256) {
      rec_status st = rec_timing_resolve(ctx);
      if (st != REC_OK) return st;
    }
    if (ctx->ev_used == ctx->ev.size()) {
      hipEvent_t a, b;
      REC_HIP(hipEventCreate(&a));
      REC_HIP(hipEventCreate(&b));
      ctx->ev.push_back({a, b});
    }
    REC_HIP(hipEventRecord(ctx->ev[ctx->ev_used].first, ctx->stream));
  }
  const ScoreScratch ss{ctx->scr_queue, ctx->counter + 13, ctx->scr_qcap, ctx->err_flag, ctx->work, false};
  rec_status st = ctx->fp32
                      ? launch_score_r<float>(ctx, P, I, J, Smap, slot, owned, gain_out, w_out, cache, ss)
                      : launch_score_r<double>(ctx, P, I, J, Smap, slot, owned, gain_out, w_out, cache, ss);
  if (ctx->timing && st == REC_OK) {
    REC_HIP(hipEventRecord(ctx->ev[ctx->ev_used].second, ctx->stream));
    ++ctx->ev_used;
    ++ctx->score_launches;
    ctx->score_pairs += P;
  }
  return st;
}
}  // namespace

rec_status rec_launch_update_chains(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                                    const uint64_t* key, const uint32_t* len, const int32_t* cpair,
                                    int64_t n, int64_t* head, uint8_t* done, double* dw) {
  if (m <= 0 || n <= 0) return REC_OK;
  return ctx->fp32 ? launch_chains_r<float>(ctx, m, I, J, key, len, cpair, n, head, done, dw)
                   : launch_chains_r<double>(ctx, m, I, J, key, len, cpair, n, head, done, dw);
}

namespace {
template <class R, int MODEL>
rec_status launch_cd_m(rec_ctx* ctx, int64_t r, int64_t n, double* acc, int64_t* changes) {
  const int64_t waves = n / 2;
  const int64_t blocks = std::min<int64_t>((waves * REC_WAVE + 255) / 256, 256 * 8);
#define REC_CD(NPL)                                                                               \
  hipLaunchKernelGGL((k_cd_round<R, NPL, MODEL>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, \
                     ctx->F, ctx->W, ctx->cfg.lambda, r, n, acc, changes, ctx->err_flag)
  switch (ctx->F.npl) {
    case 1: REC_CD(1); break;
    case 2: REC_CD(2); break;
    case 4: REC_CD(4); break;
    case 8: REC_CD(8); break;
    case 16: REC_CD(16); break;
    case 32: REC_CD(32); break;
    default: ctx->err = "unsupported sample count"; return REC_E_INVAL;
  }
#undef REC_CD
  return hipGetLastError() == hipSuccess ? REC_OK : REC_E_HIP;
}

template <class R>
rec_status launch_cd_r(rec_ctx* ctx, int64_t r, int64_t n, double* acc, int64_t* changes) {
  switch (ctx->cfg.model) {
    case REC_ISING: return launch_cd_m<R, REC_ISING>(ctx, r, n, acc, changes);
    case REC_GAUSS: return launch_cd_m<R, REC_GAUSS>(ctx, r, n, acc, changes);
    case REC_KINETIC: return launch_cd_m<R, REC_KINETIC>(ctx, r, n, acc, changes);
  }
  return REC_E_INVAL;
}
}  // namespace

rec_status rec_launch_cd_round(rec_ctx* ctx, int64_t r, int64_t n, double* acc, int64_t* changes) {
  return ctx->fp32 ? launch_cd_r<float>(ctx, r, n, acc, changes) : launch_cd_r<double>(ctx, r, n, acc, changes);
}

rec_status rec_launch_update_round(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J,
                                   const int32_t* ready, const int64_t* nready, uint8_t* done,
                                   double* dw, int32_t* depth, int32_t round) {
  if (m <= 0) return REC_OK;
  return ctx->fp32 ? launch_update_r<float>(ctx, m, I, J, ready, nready, done, dw, depth, round)
                   : launch_update_r<double>(ctx, m, I, J, ready, nready, done, dw, depth, round);
}

rec_status rec_launch_update_flow(rec_ctx* ctx, int64_t m, const int32_t* I, const int32_t* J, const int32_t* pred,
                                  uint8_t* done, double* dw, int32_t* depth, int64_t* ticket, int64_t* rounds,
                                  int64_t* abort_flag, int64_t spin_limit) {
  if (m <= 0) return REC_OK;
  return ctx->fp32 ? launch_update_flow_r<float>(ctx, m, I, J, pred, done, dw, depth, ticket, rounds, abort_flag,
                                                 spin_limit)
                   : launch_update_flow_r<double>(ctx, m, I, J, pred, done, dw, depth, ticket, rounds, abort_flag,
                                                  spin_limit);
}
