// Reference oracle for greedy coordinate descent (GCD) network reconstruction,
// following T. P. Peixoto, "Scalable network reconstruction in subquadratic
// time" (arXiv 2401.01404).
//
// TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
// whose job is to be obviously correct.  Only the test suite, the smoke check
// and the CPU-baseline leg of the benchmark may load it; the GPU library
// never calls, links or includes anything from here, and nothing here comes
// from the GPU library.  OpenMP is used only across independent pairs or
// nodes; every coordinate update is sequential.
//
// What it computes (paper references in brackets):
//   * the log pseudolikelihood objective of the Ising model [App. A, Ising
//     pseudolikelihood], of the Gaussian model [App. A, Gaussian
//     pseudolikelihood, theta_i = 1/sqrt(W_ii)] and of a kinetic Ising time
//     series [Sec. 2, Markov product form], plus the Laplace prior
//     [App. A, L1 prior];
//   * the edge score d(i,j) = -max_{W_ij} pi(W) [Alg. 2, function D], kept as
//     the equivalent nonnegative gain max_w pi(W_ij <- w) - pi(W);
//   * exhaustive scoring, FindBest [Alg. 3] with exact KNN or with NNDescent
//     [Alg. 4], the GCD sweep [Alg. 2], the CD sweep [Alg. 1] and the field
//     updates theta [App. A, "updated alongside W"].
//
// Readings of points the paper leaves open (each one is listed with its
// reason in the design notes of the repository):
//   R1 gain = max pi - pi(W) >= 0 ranks like d = -max pi.
//   R2 the 1-D argmax is found by Newton steps safeguarded by bisection on a
//      bracket of the (monotone) derivative; the maximiser is unique because
//      the 1-D problem is concave, so the solver does not change the result.
//   R3 ties: pairs rank by (gain desc, min(i,j) asc, max(i,j) asc); a node's
//      neighbour list by (gain desc, j asc); directed edges (i->j) by (gain
//      desc, min, max, i asc); kinetic ordered pairs by (gain desc, i, j).
//   R4 m = round-half-up(kappa N), at least 1; k = ceil(4m/|S|) clamped to
//      |S|-1.
//   R5 NNDescent: random initial lists by Floyd's sampling from SplitMix64
//      counters; one iteration replaces every list at once by the top-k of
//      (old list + second neighbours), the order-independent form of the
//      per-node update; U(j) = out(j) + at most k in-neighbours of j, those
//      with the smallest (32-bit counter hash, index); stop when
//      changes/(k|S|) < eps or at 2 ceil(log_{2k}|S|) + 10 iterations.
//   R6 theta is refitted for every node after each sweep's W updates; its
//      initial value is the W = 0 optimum; it is clamped to [-8, 8].
//   R7 kinetic Ising: P(x_t | x_{t-1}) = prod_i exp(x_{i,t} h_{i,t-1}) /
//      2cosh(h_{i,t-1}), W directed, pairs are ordered (i <- j).  FindBest
//      [Alg. 3] needs a symmetric d: it runs over unordered pairs scored by
//      max(gain(i <- j), gain(j <- i)) and the best m directed pairs are
//      taken from both directions of the m unordered pairs it returns (exact
//      when the KNN lists are exact, since at most m unordered pairs reach the
//      m-th best directed gain).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

enum Model { ISING = 0, GAUSS = 1, KINETIC = 2 };
constexpr double THETA_MAX = 8.0;

// ------------------------------------------------------------ numerics ----

// log cosh x, accurate for small and large |x|.
double lcosh(double x) {
  double a = std::fabs(x);
  if (a < 1.0) {
    double s = std::sinh(0.5 * x);
    return std::log1p(2.0 * s * s);           // cosh x = 1 + 2 sinh^2(x/2)
  }
  return a + std::log1p(std::exp(-2.0 * a)) - std::log(2.0);
}

// lcosh(a + d) - lcosh(a), without cancellation when d is small.
double dlcosh(double a, double d) {
  double p = std::tanh(a) * std::tanh(d);
  if (p > -0.5) return lcosh(d) + std::log1p(p);   // cosh(a+d) = cosh a cosh d (1 + tanh a tanh d)
  return lcosh(a + d) - lcosh(a);
}

double sgn(double x) { return (x > 0) - (x < 0); }

// Root of a decreasing function phi on [lo, hi] with phi(lo) > 0 > phi(hi):
// Newton steps (dphi < 0 supplied by the callback) kept inside the bracket,
// bisection otherwise.  Returns the point where the bracket closed.
template <class F>
double safe_root(F&& f, double lo, double hi) {
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    double fx, dfx;
    f(x, fx, dfx);
    if (fx == 0.0) return x;
    if (fx > 0) lo = x; else hi = x;
    double xn = (dfx < 0) ? x - fx / dfx : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 1e-16 * std::max(1.0, std::fabs(x)) ||
        hi - lo <= 4e-16 * std::max(1.0, std::fabs(lo) + std::fabs(hi)))
      return xn;
    x = xn;
  }
  return x;
}

// ------------------------------------------------------------- problem ----

struct Problem {
  int model;
  int64_t N, M;                  // M = samples (kinetic: transitions)
  std::vector<double> in;        // N x M: x_{j,m}      (kinetic: x_{j,t-1})
  std::vector<double> out;       // N x M: target x_{i,m} (kinetic: x_{i,t})
  double lambda;
  std::map<std::pair<int, int>, double> W;   // symmetric: key (min,max); kinetic: (i, j)
  std::vector<double> theta;     // Ising/kinetic: field; Gaussian: theta_i = 1/sqrt(W_ii)
  std::vector<double> msum;      // N x M: m_{i,m} = sum_{j != i} W_ij in_{j,m}
  std::vector<double> sq;        // Gaussian: ||x_i||^2
  int dist = 0;                  // search distance: 0 the exact gain, 1 the absolute gradient

  double X(int64_t i, int64_t m) const { return in[i * M + m]; }
  double Y(int64_t i, int64_t m) const { return out[i * M + m]; }
  std::pair<int, int> key(int i, int j) const {
    if (model == KINETIC) return {i, j};
    return {std::min(i, j), std::max(i, j)};
  }
  double w(int i, int j) const {
    auto it = W.find(key(i, j));
    return it == W.end() ? 0.0 : it->second;
  }
};

// m_{i,m} from scratch [App. A: "keeping track of the weighted sum of the
// neighbors m_i"].
void rebuild_msum(Problem& P) {
  std::fill(P.msum.begin(), P.msum.end(), 0.0);
  for (auto& kv : P.W) {
    int i = kv.first.first, j = kv.first.second;
    double w = kv.second;
    if (w == 0.0) continue;
    for (int64_t m = 0; m < P.M; ++m) P.msum[i * P.M + m] += w * P.X(j, m);
    if (P.model != KINETIC)
      for (int64_t m = 0; m < P.M; ++m) P.msum[j * P.M + m] += w * P.X(i, m);
  }
}

// ----------------------------------------------------------- objective ----

// Log pseudolikelihood of node i's conditional(s).
//   Ising [App. A]:  sum_m x_im h_im - log(2 cosh h_im),  h = theta_i + m_i
//   kinetic [Sec. 2 Markov form]: the same with target x_{i,t}, field from x_{t-1}
//   Gaussian [App. A]: sum_m -(x_im + theta_i^2 m_im)^2 / (2 theta_i^2)
//                      - log theta_i - log(2 pi)/2
double node_loglik(const Problem& P, int64_t i) {
  double s = 0.0;
  if (P.model == GAUSS) {
    double v = P.theta[i] * P.theta[i];
    for (int64_t m = 0; m < P.M; ++m) {
      double r = P.Y(i, m) + v * P.msum[i * P.M + m];
      s += -r * r / (2.0 * v);
    }
    s += P.M * (-std::log(P.theta[i]) - 0.5 * std::log(2.0 * M_PI));
    return s;
  }
  for (int64_t m = 0; m < P.M; ++m) {
    double h = P.theta[i] + P.msum[i * P.M + m];
    s += P.Y(i, m) * h - lcosh(h) - std::log(2.0);
  }
  return s;
}

// log pi(W) up to the constant of the Laplace prior [App. A]:
// sum_i node_loglik - lambda * sum_{i<j} |W_ij| (kinetic: sum over i != j).
double objective(const Problem& P) {
  double L = 0.0;
#pragma omp parallel for reduction(+ : L) schedule(static)
  for (int64_t i = 0; i < P.N; ++i) L += node_loglik(P, i);
  double pen = 0.0;
  for (auto& kv : P.W) pen += std::fabs(kv.second);
  return L - P.lambda * pen;
}

// ------------------------------------------------------------ pair gain ---

// Smooth part F(delta) of the objective change when W_ij moves from w0 to
// w0 + delta, and its first two derivatives.  For the Ising model both
// conditionals of i and j change [App. A]; for the kinetic model only row i
// (target i, source j); the Gaussian case is handled in closed form below.
struct Smooth {
  const Problem& P;
  int i, j;
  void d12(double delta, double& f1, double& f2) const {
    double a1 = 0.0, a2 = 0.0;
    for (int64_t m = 0; m < P.M; ++m) {
      double hi = P.theta[i] + P.msum[i * P.M + m];
      double xj = P.X(j, m);
      double t = std::tanh(hi + delta * xj);
      a1 += xj * (P.Y(i, m) - t);
      a2 -= 1.0 - t * t;
      if (P.model == ISING) {
        double hj = P.theta[j] + P.msum[j * P.M + m];
        double xi = P.X(i, m);
        double u = std::tanh(hj + delta * xi);
        a1 += xi * (P.Y(j, m) - u);
        a2 -= 1.0 - u * u;
      }
    }
    f1 = a1;
    f2 = a2;
  }
  double f(double delta) const {
    double s = 0.0;
    for (int64_t m = 0; m < P.M; ++m) {
      double hi = P.theta[i] + P.msum[i * P.M + m];
      double xj = P.X(j, m);
      s += delta * xj * P.Y(i, m) - dlcosh(hi, delta * xj);
      if (P.model == ISING) {
        double hj = P.theta[j] + P.msum[j * P.M + m];
        double xi = P.X(i, m);
        s += delta * xi * P.Y(j, m) - dlcosh(hj, delta * xi);
      }
    }
    return s;
  }
};

// gain(i,j) = max_w [pi(W_ij <- w) - pi(W)] >= 0 and its argmax w*
// [Alg. 2, function D; Alg. 1 step (1)].  The objective restricted to one
// coordinate is F(w - w0) - lambda |w| + lambda |w0| with F concave, so w* is
// 0 when |F'(-w0)| <= lambda, else the root of F'(w - w0) = s lambda on the
// side s = sign F'(-w0).
void pair_gain(const Problem& P, int i, int j, double* gain, double* wopt) {
  // symmetric models: evaluate in canonical order so that d(i,j) and d(j,i)
  // are the same floating-point number
  if (P.model != KINETIC && i > j) std::swap(i, j);
  double w0 = P.w(i, j);
  double lam = P.lambda;
  if (P.model == GAUSS) {
    // Closed form: with r_i = x_i + theta_i^2 m_i the change of the two
    // conditionals is a delta - b delta^2 / 2 with
    //   a = -(r_i . x_j + r_j . x_i),  b = theta_i^2 ||x_j||^2 + theta_j^2 ||x_i||^2.
    double vi = P.theta[i] * P.theta[i], vj = P.theta[j] * P.theta[j];
    double a = 0.0;
    for (int64_t m = 0; m < P.M; ++m) {
      double ri = P.Y(i, m) + vi * P.msum[i * P.M + m];
      double rj = P.Y(j, m) + vj * P.msum[j * P.M + m];
      a -= ri * P.X(j, m) + rj * P.X(i, m);
    }
    double b = vi * P.sq[j] + vj * P.sq[i];
    // maximise a (w - w0) - b (w - w0)^2 / 2 - lambda |w|: soft threshold
    double z = w0 + a / b;
    double ws = sgn(z) * std::max(std::fabs(z) - lam / b, 0.0);
    double d = ws - w0;
    *wopt = ws;
    *gain = a * d - 0.5 * b * d * d - lam * (std::fabs(ws) - std::fabs(w0));
    return;
  }
  Smooth F{P, i, j};
  double g0, h0;
  F.d12(-w0, g0, h0);                      // derivative at w = 0
  double ws;
  if (std::fabs(g0) <= lam) {
    ws = 0.0;
  } else {
    double s = sgn(g0);
    auto phi = [&](double w, double& fx, double& dfx) {
      double f1, f2;
      F.d12(w - w0, f1, f2);
      fx = s * (f1 - s * lam);             // decreasing in s*w
      dfx = f2;                            // d/d(s w) of s*(f1 - s lam) = f2
    };
    // bracket in u = s*w >= 0: phi(0) > 0; double until phi < 0
    auto phis = [&](double u, double& fx, double& dfx) { phi(s * u, fx, dfx); };
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
      double fx, dfx;
      phis(hi, fx, dfx);
      if (fx < 0) break;
      lo = hi;
      hi *= 2.0;
    }
    ws = s * safe_root(phis, lo, hi);
  }
  *wopt = ws;
  *gain = F.f(ws - w0) - lam * (std::fabs(ws) - std::fabs(w0));
}

// Gradient as distance [Appendix, "Gradient as distance"]: the absolute
// derivative of the objective with respect to W_ij at the current state,
// taken as the paper takes it for L1-penalised objectives, by a central
// difference: away from the kink (w0 != 0) it is F'(w0) - lambda sign(w0);
// at w0 = 0 the two one-sided penalty terms cancel and it is F'(0).  The
// score is its absolute value (larger = better, as for the gain).
double pair_grad(const Problem& P, int i, int j) {
  if (P.model != KINETIC && i > j) std::swap(i, j);
  const double w0 = P.w(i, j);
  double f1;
  if (P.model == GAUSS) {
    // F(delta) = a delta - b delta^2 / 2 around the current state
    const double vi = P.theta[i] * P.theta[i], vj = P.theta[j] * P.theta[j];
    double a = 0.0;
    for (int64_t m = 0; m < P.M; ++m)
      a -= (P.Y(i, m) + vi * P.msum[i * P.M + m]) * P.X(j, m) +
           (P.Y(j, m) + vj * P.msum[j * P.M + m]) * P.X(i, m);
    f1 = a;
  } else {
    double f2;
    Smooth{P, i, j}.d12(0.0, f1, f2);
  }
  return std::fabs(w0 == 0.0 ? f1 : f1 - P.lambda * sgn(w0));
}

// The search score of a pair under the problem's distance.
double pair_dist(const Problem& P, int i, int j) {
  if (P.dist == 1) return pair_grad(P, i, j);
  double g, w;
  pair_gain(P, i, j, &g, &w);
  return g;
}

// -------------------------------------------------------------- updates ---

// W_ij <- w, keeping m_i (and m_j) current [App. A].
void set_w(Problem& P, int i, int j, double w) {
  double w0 = P.w(i, j);
  double d = w - w0;
  if (d != 0.0) {
    for (int64_t m = 0; m < P.M; ++m) P.msum[i * P.M + m] += d * P.X(j, m);
    if (P.model != KINETIC)
      for (int64_t m = 0; m < P.M; ++m) P.msum[j * P.M + m] += d * P.X(i, m);
  }
  if (w == 0.0) P.W.erase(P.key(i, j));
  else P.W[P.key(i, j)] = w;
}

// theta_i <- argmax of node i's conditional(s) [App. A: "we update alongside W"].
//   Ising / kinetic: root of sum_m (y_im - tanh(theta + m_im)) = 0, clamped.
//   Gaussian: v = theta_i^2 solves C v^2 + M v - A = 0 with A = sum x_im^2,
//   C = sum m_im^2 (v = A / M when C = 0).
void theta_update(Problem& P) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < P.N; ++i) {
    if (P.model == GAUSS) {
      double A = 0.0, C = 0.0;
      for (int64_t m = 0; m < P.M; ++m) {
        A += P.Y(i, m) * P.Y(i, m);
        C += P.msum[i * P.M + m] * P.msum[i * P.M + m];
      }
      double v = C > 0 ? (-double(P.M) + std::sqrt(double(P.M) * P.M + 4.0 * A * C)) / (2.0 * C)
                       : A / P.M;
      P.theta[i] = std::sqrt(v);
      continue;
    }
    auto phi = [&](double th, double& fx, double& dfx) {
      double a = 0.0, b = 0.0;
      for (int64_t m = 0; m < P.M; ++m) {
        double t = std::tanh(th + P.msum[i * P.M + m]);
        a += P.Y(i, m) - t;
        b -= 1.0 - t * t;
      }
      fx = a;
      dfx = b;
    };
    double f1, f2;
    phi(THETA_MAX, f1, f2);
    if (f1 >= 0) { P.theta[i] = THETA_MAX; continue; }
    phi(-THETA_MAX, f1, f2);
    if (f1 <= 0) { P.theta[i] = -THETA_MAX; continue; }
    P.theta[i] = safe_root(phi, -THETA_MAX, THETA_MAX);
  }
}

// ----------------------------------------------------------- orderings ----

struct Pair { int i, j; double g; };

// undirected pairs (and kinetic ordered pairs): gain desc, then indices
bool pair_less(const Problem& P, const Pair& a, const Pair& b) {
  if (a.g != b.g) return a.g > b.g;
  if (P.model == KINETIC) {
    if (a.i != b.i) return a.i < b.i;
    return a.j < b.j;
  }
  int a0 = std::min(a.i, a.j), a1 = std::max(a.i, a.j);
  int b0 = std::min(b.i, b.j), b1 = std::max(b.i, b.j);
  if (a0 != b0) return a0 < b0;
  return a1 < b1;
}

// directed edges i->j of a KNN graph: gain desc, min, max, then i
bool edge_less(const Pair& a, const Pair& b) {
  if (a.g != b.g) return a.g > b.g;
  int a0 = std::min(a.i, a.j), a1 = std::max(a.i, a.j);
  int b0 = std::min(b.i, b.j), b1 = std::max(b.i, b.j);
  if (a0 != b0) return a0 < b0;
  if (a1 != b1) return a1 < b1;
  return a.i < b.i;
}

// ----------------------------------------------------------- RNG (R5) -----

uint64_t mix64(uint64_t z) {   // SplitMix64 output function (Steele et al. 2014)
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
uint64_t ctr(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(mix64(seed) ^ stream) ^ a) ^ b);
}
uint64_t below(uint64_t r, uint64_t bound) {   // floor(r * bound / 2^64)
  return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}
constexpr uint64_t STREAM_INIT = 5, STREAM_CAP = 6;

// ------------------------------------------------------------------ KNN ---

struct Nb { int j; double g; };
bool nb_less(const Nb& a, const Nb& b) {
  if (a.g != b.g) return a.g > b.g;
  return a.j < b.j;
}

// Search score of an unordered pair.  Symmetric models: the gain.  Kinetic
// model (directed W, R14): FindBest runs over unordered pairs {i, j} scored by
// max(gain(i <- j), gain(j <- i)); the best m directed pairs are then taken
// from both directions of the m pairs found (see find_best_kinetic).
struct ScoreFn {
  const Problem& P;
  double operator()(int i, int j) const {
    double g = pair_dist(P, i, j);
    if (P.model == KINETIC) g = std::max(g, pair_dist(P, j, i));
    return g;
  }
};

// Exact k nearest neighbours of each node of S within S.
std::vector<std::vector<Nb>> knn_exact(const Problem& P, const std::vector<int>& S, int k) {
  int64_t n = S.size();
  std::vector<std::vector<Nb>> G(n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < n; ++a) {
    std::vector<Nb> all;
    for (int64_t b = 0; b < n; ++b)
      if (b != a) all.push_back({S[b], ScoreFn{P}(S[a], S[b])});
    std::sort(all.begin(), all.end(), nb_less);
    all.resize(std::min<int64_t>(k, all.size()));
    G[a] = all;
  }
  return G;
}

// Random initial list of node a (local index) [Alg. 4, first step]:
// k distinct local indices != a, Floyd's algorithm over the n-1 others.
std::vector<int> knn_init_local(int64_t n, int64_t a, int k, uint64_t seed, int level, int gid) {
  std::vector<int> chosen;
  std::unordered_set<int64_t> has;
  uint64_t tag = ((uint64_t)level << 32) | (uint32_t)gid;
  for (int64_t t = (n - 1) - k; t <= n - 2; ++t) {
    int64_t v = (int64_t)below(ctr(seed, STREAM_INIT, tag, (uint64_t)t), (uint64_t)(t + 1));
    int64_t pick = has.count(v) ? t : v;
    has.insert(pick);
    chosen.push_back((int)(pick < a ? pick : pick + 1));
  }
  return chosen;
}

struct KnnStats { int iters; int64_t evals; };

// NNDescent [Alg. 4] in its order-independent form (R5).  Returns lists in
// local order of S (global ids inside).
std::vector<std::vector<Nb>> knn_nndescent(const Problem& P, const std::vector<int>& S, int k,
                                           uint64_t seed, int level, double eps, int max_iter,
                                           KnnStats* st) {
  int64_t n = S.size();
  std::vector<int64_t> loc(P.N, -1);
  for (int64_t a = 0; a < n; ++a) loc[S[a]] = a;
  std::vector<std::vector<Nb>> G(n);
  int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
  for (int64_t a = 0; a < n; ++a) {
    std::vector<int> init = knn_init_local(n, a, k, seed, level, S[a]);
    for (int b : init) { G[a].push_back({S[b], ScoreFn{P}(S[a], S[b])}); ++evals; }
    std::sort(G[a].begin(), G[a].end(), nb_less);
  }
  if (max_iter <= 0) {
    int lg = 0;
    for (double c = 1; c < n; c *= 2.0 * k) ++lg;   // ceil(log_{2k} n)
    max_iter = 2 * lg + 10;
  }
  int it = 0;
  for (; it < max_iter; ++it) {
    // U = undirected version of G with at most k in-neighbours per node
    std::vector<std::vector<std::pair<uint64_t, int>>> in(n);
    for (int64_t a = 0; a < n; ++a)
      for (auto& e : G[a]) {
        int64_t b = loc[e.j];
        uint64_t h = ctr(seed, STREAM_CAP, ((uint64_t)level << 32) | (uint32_t)it,
                         ((uint64_t)(uint32_t)S[a] << 32) | (uint32_t)e.j) >> 32;
        in[b].push_back({h, (int)a});
      }
    std::vector<std::vector<int>> U(n);
    for (int64_t b = 0; b < n; ++b) {
      std::sort(in[b].begin(), in[b].end());
      std::set<int> s;
      for (auto& e : G[b]) s.insert((int)loc[e.j]);
      for (size_t c = 0; c < in[b].size() && (int)c < k; ++c) s.insert(in[b][c].second);
      U[b].assign(s.begin(), s.end());
    }
    std::vector<std::vector<Nb>> G2(n);
    int64_t delta = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : delta, evals)
    for (int64_t a = 0; a < n; ++a) {
      std::set<int> cur;
      for (auto& e : G[a]) cur.insert(e.j);
      std::set<int> cand;
      for (int b : U[a])
        for (int c : U[b]) {
          int v = S[c];
          if (c == a || cur.count(v)) continue;
          cand.insert(v);
        }
      std::vector<Nb> all = G[a];
      for (int v : cand) { all.push_back({v, ScoreFn{P}(S[a], v)}); ++evals; }
      std::sort(all.begin(), all.end(), nb_less);
      all.resize(std::min<size_t>(k, all.size()));
      for (auto& e : all) delta += cur.count(e.j) ? 0 : 1;
      G2[a] = all;
    }
    G.swap(G2);
    if ((double)delta < eps * (double)k * (double)n) { ++it; break; }
  }
  if (st) { st->iters = it; st->evals += evals; }
  return G;
}

// ------------------------------------------------------------- FindBest ---

struct FBStats { int levels; int iters; int64_t evals; int64_t level_n[64]; int level_k[64]; };

// All pairs of S, best first.
std::vector<Pair> exhaustive(const Problem& P, const std::vector<int>& S) {
  int64_t n = S.size();
  std::vector<std::vector<Pair>> rows(n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < n; ++a) {
    int64_t b0 = P.model == KINETIC ? 0 : a + 1;
    for (int64_t b = b0; b < n; ++b) {
      if (b == a) continue;
      const double g = pair_dist(P, S[a], S[b]);
      if (P.model == KINETIC) rows[a].push_back({S[a], S[b], g});
      else rows[a].push_back({std::min(S[a], S[b]), std::max(S[a], S[b]), g});
    }
  }
  std::vector<Pair> all;
  for (auto& r : rows) all.insert(all.end(), r.begin(), r.end());
  std::sort(all.begin(), all.end(), [&](const Pair& x, const Pair& y) { return pair_less(P, x, y); });
  return all;
}

// All unordered pairs of S under the search score, best first (base case of
// FindBest; for the symmetric models this is exhaustive()).
std::vector<Pair> exhaustive_sym(const Problem& P, const std::vector<int>& S) {
  if (P.model != KINETIC) return exhaustive(P, S);
  int64_t n = S.size();
  std::vector<std::vector<Pair>> rows(n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a + 1; b < n; ++b)
      rows[a].push_back({S[a], S[b], ScoreFn{P}(S[a], S[b])});
  std::vector<Pair> all;
  for (auto& r : rows) all.insert(all.end(), r.begin(), r.end());
  std::sort(all.begin(), all.end(), [](const Pair& x, const Pair& y) {
    if (x.g != y.g) return x.g > y.g;
    if (x.i != y.i) return x.i < y.i;
    return x.j < y.j;
  });
  return all;
}

// FindBest(m, S, d) [Alg. 3] for the symmetric models, written as a loop over
// recursion levels that accumulates D in a pool and returns its best m.
// mode 1: exact KNN; mode 2: NNDescent.
std::vector<Pair> find_best(const Problem& P, int64_t m, int mode, uint64_t seed, double eps,
                            int max_iter, FBStats* st) {
  std::vector<int> S(P.N);
  for (int64_t i = 0; i < P.N; ++i) S[i] = (int)i;
  std::map<std::pair<int, int>, double> pool;
  int level = 0;
  if (st) { st->levels = 0; st->iters = 0; st->evals = 0; }
  while (true) {
    int64_t n = S.size();
    if (st && level < 64) st->level_n[level] = n;
    if (n * n <= 4 * m || n < 2) {         // base case: exhaustive over S
      for (auto& p : exhaustive_sym(P, S)) pool[{p.i, p.j}] = p.g;
      if (st) { st->evals += n * (n - 1) / 2; if (level < 64) st->level_k[level] = 0; }
      ++level;
      break;
    }
    int k = (int)std::min<int64_t>((4 * m + n - 1) / n, n - 1);
    if (st && level < 64) st->level_k[level] = k;
    std::vector<std::vector<Nb>> G;
    if (mode == 1) {
      G = knn_exact(P, S, k);
      if (st) st->evals += n * (n - 1);
    } else {
      KnnStats ks{0, 0};
      G = knn_nndescent(P, S, k, seed, level, eps, max_iter, &ks);
      if (st) { st->iters += ks.iters; st->evals += ks.evals; }
    }
    // D+ = the 2m best directed edges of G; D = their undirected pairs
    std::vector<Pair> E;
    for (int64_t a = 0; a < n; ++a)
      for (auto& e : G[a]) E.push_back({S[a], e.j, e.g});
    std::sort(E.begin(), E.end(), edge_less);
    E.resize(std::min<int64_t>(2 * m, E.size()));
    std::set<std::pair<int, int>> D;
    for (auto& e : E) {
      auto key = std::make_pair(std::min(e.i, e.j), std::max(e.i, e.j));
      D.insert(key);
      pool[key] = e.g;
    }
    // S' = nodes all of whose out-neighbours are paired with them in D
    std::vector<int> S2;
    for (int64_t a = 0; a < n; ++a) {
      bool all = true;
      for (auto& e : G[a])
        if (!D.count({std::min(S[a], e.j), std::max(S[a], e.j)})) { all = false; break; }
      if (all) S2.push_back(S[a]);
    }
    ++level;
    if (S2.size() == S.size()) break;      // cannot happen when n^2 > 4m; guard only
    S.swap(S2);
  }
  if (st) st->levels = level;
  std::vector<Pair> res;
  for (auto& kv : pool) res.push_back({kv.first.first, kv.first.second, kv.second});
  // unordered pairs: (gain desc, min, max)
  std::sort(res.begin(), res.end(), [](const Pair& x, const Pair& y) {
    if (x.g != y.g) return x.g > y.g;
    if (x.i != y.i) return x.i < y.i;
    return x.j < y.j;
  });
  if ((int64_t)res.size() > m) res.resize(m);
  if (P.model != KINETIC) return res;
  // kinetic: the best m directed pairs among both directions of the m found
  std::vector<Pair> dir;
  for (auto& p : res)
    for (int d = 0; d < 2; ++d) {
      int i = d ? p.j : p.i, j = d ? p.i : p.j;
      dir.push_back({i, j, pair_dist(P, i, j)});
    }
  std::sort(dir.begin(), dir.end(), [&](const Pair& x, const Pair& y) { return pair_less(P, x, y); });
  if ((int64_t)dir.size() > m) dir.resize(m);
  return dir;
}

}  // namespace

// ================================================================= C ABI ==

extern "C" {

// Create a problem.  xtype 0: int8 +-1; 1: float32.  X is node-major with
// row stride ldx; for the kinetic model X has M+1 columns (states t=0..M).
// theta starts at the W = 0 optimum (R6).
void* orc_create(int model, int64_t N, int64_t M, int xtype, const void* X, int64_t ldx,
                 double lambda) {
  Problem* P = new Problem();
  P->model = model;
  P->N = N;
  P->M = M;
  P->lambda = lambda;
  P->in.assign(N * M, 0.0);
  P->out.assign(N * M, 0.0);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t m = 0; m < M; ++m) {
      auto get = [&](int64_t col) {
        return xtype == 0 ? (double)((const int8_t*)X)[i * ldx + col]
                          : (double)((const float*)X)[i * ldx + col];
      };
      if (model == KINETIC) {
        P->in[i * M + m] = get(m);
        P->out[i * M + m] = get(m + 1);
      } else {
        P->in[i * M + m] = P->out[i * M + m] = get(m);
      }
    }
  P->msum.assign(N * M, 0.0);
  P->theta.assign(N, model == GAUSS ? 1.0 : 0.0);
  P->sq.assign(N, 0.0);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t m = 0; m < M; ++m) P->sq[i] += P->in[i * M + m] * P->in[i * M + m];
  theta_update(*P);
  return P;
}

void orc_destroy(void* h) { delete (Problem*)h; }

// Replace W (and theta when given); entries with w == 0 are dropped.
void orc_set_model(void* h, int64_t nnz, const int32_t* ei, const int32_t* ej, const double* w,
                   const double* theta) {
  Problem& P = *(Problem*)h;
  P.W.clear();
  for (int64_t e = 0; e < nnz; ++e)
    if (w[e] != 0.0) P.W[P.key(ei[e], ej[e])] = w[e];
  if (theta) for (int64_t i = 0; i < P.N; ++i) P.theta[i] = theta[i];
  rebuild_msum(P);
}

int64_t orc_get_model(void* h, int64_t cap, int32_t* ei, int32_t* ej, double* w, double* theta) {
  Problem& P = *(Problem*)h;
  int64_t c = 0;
  for (auto& kv : P.W) {
    if (c < cap) { ei[c] = kv.first.first; ej[c] = kv.first.second; w[c] = kv.second; }
    ++c;
  }
  if (theta) for (int64_t i = 0; i < P.N; ++i) theta[i] = P.theta[i];
  return c;
}

double orc_objective(void* h) { return objective(*(Problem*)h); }
double orc_node_loglik(void* h, int64_t i) { return node_loglik(*(Problem*)h, i); }

// fields h_{i,m} = theta_i + m_{i,m} (Gaussian: residual x_im + theta_i^2 m_im)
void orc_fields(void* h, double* H) {
  Problem& P = *(Problem*)h;
  for (int64_t i = 0; i < P.N; ++i)
    for (int64_t m = 0; m < P.M; ++m) {
      double ms = P.msum[i * P.M + m];
      H[i * P.M + m] = P.model == GAUSS ? P.Y(i, m) + P.theta[i] * P.theta[i] * ms : P.theta[i] + ms;
    }
}

void orc_theta_update(void* h) { theta_update(*(Problem*)h); }

void orc_score_pairs(void* h, int64_t n, const int32_t* I, const int32_t* J, double* gain,
                     double* wopt) {
  Problem& P = *(Problem*)h;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) {
    double g, w;
    pair_gain(P, I[p], J[p], &g, &w);
    gain[p] = g;
    if (wopt) wopt[p] = w;
  }
}

// Derivative of the smooth part at w (for KKT checks): dF/dW_ij at W_ij = w.
double orc_pair_deriv(void* h, int32_t i, int32_t j, double w) {
  Problem& P = *(Problem*)h;
  if (P.model == GAUSS) {
    double vi = P.theta[i] * P.theta[i], vj = P.theta[j] * P.theta[j];
    double a = 0.0;
    for (int64_t m = 0; m < P.M; ++m) {
      a -= (P.Y(i, m) + vi * P.msum[i * P.M + m]) * P.X(j, m) +
           (P.Y(j, m) + vj * P.msum[j * P.M + m]) * P.X(i, m);
    }
    double b = vi * P.sq[j] + vj * P.sq[i];
    return a - b * (w - P.w(i, j));
  }
  Smooth F{P, i, j};
  double f1, f2;
  F.d12(w - P.w(i, j), f1, f2);
  return f1;
}

// Best m pairs.  mode 0: exhaustive; 1: FindBest with exact KNN; 2: FindBest
// with NNDescent.  Writes up to m pairs best first; returns the count.
// stats (may be null): [levels, nnd_iters, evals, n_0, k_0, n_1, k_1, ...].
int64_t orc_find_best(void* h, int64_t m, int mode, uint64_t seed, double eps, int max_iter,
                      int32_t* oi, int32_t* oj, double* og, int64_t* stats) {
  Problem& P = *(Problem*)h;
  std::vector<Pair> res;
  FBStats st{};
  if (mode == 0) {
    std::vector<int> S(P.N);
    for (int64_t i = 0; i < P.N; ++i) S[i] = (int)i;
    res = exhaustive(P, S);
    if ((int64_t)res.size() > m) res.resize(m);
    st.levels = 0;
    st.evals = P.model == KINETIC ? P.N * (P.N - 1) : P.N * (P.N - 1) / 2;
  } else {
    res = find_best(P, m, mode, seed, eps, max_iter, &st);
  }
  for (size_t c = 0; c < res.size(); ++c) { oi[c] = res[c].i; oj[c] = res[c].j; og[c] = res[c].g; }
  if (stats) {
    stats[0] = st.levels; stats[1] = st.iters; stats[2] = st.evals;
    for (int l = 0; l < std::min(st.levels, 30); ++l) { stats[3 + 2 * l] = st.level_n[l]; stats[4 + 2 * l] = st.level_k[l]; }
  }
  return (int64_t)res.size();
}

// k-NN lists over the node subset S (global ids) at FindBest level `level`.
// mode 1: exact; 2: NNDescent.  Writes n*k (j, gain) best first per node;
// returns the number of NNDescent iterations.
int orc_knn(void* h, int64_t n, const int32_t* S, int k, int mode, uint64_t seed, int level,
            double eps, int max_iter, int32_t* oj, double* og) {
  Problem& P = *(Problem*)h;
  std::vector<int> s(S, S + n);
  KnnStats ks{0, 0};
  auto G = mode == 1 ? knn_exact(P, s, k) : knn_nndescent(P, s, k, seed, level, eps, max_iter, &ks);
  for (int64_t a = 0; a < n; ++a)
    for (int c = 0; c < k; ++c) {
      bool ok = c < (int)G[a].size();
      oj[a * k + c] = ok ? G[a][c].j : -1;
      og[a * k + c] = ok ? G[a][c].g : 0.0;
    }
  return ks.iters;
}

// Random initial KNN list (local indices) of node a in a set of n nodes.
void orc_knn_init(int64_t n, int64_t a, int k, uint64_t seed, int level, int gid, int32_t* out) {
  auto v = knn_init_local(n, a, k, seed, level, gid);
  for (int c = 0; c < k; ++c) out[c] = v[c];
}

// Apply coordinate updates to the given pairs in order [Alg. 2 loop body]:
// W_ij <- argmax with the current state.  Returns Delta = sum |W' - W|.
// check != 0: recompute the objective after every update and count updates
// that lowered it by more than 1e-12 |L| (written to *bad).
double orc_apply_updates(void* h, int64_t n, const int32_t* I, const int32_t* J, int check,
                         int64_t* bad) {
  Problem& P = *(Problem*)h;
  double delta = 0.0;
  int64_t nbad = 0;
  double L = check ? objective(P) : 0.0;
  for (int64_t p = 0; p < n; ++p) {
    double g, w;
    pair_gain(P, I[p], J[p], &g, &w);
    delta += std::fabs(w - P.w(I[p], J[p]));
    set_w(P, I[p], J[p], w);
    if (check) {
      double L2 = objective(P);
      if (L2 < L - 1e-12 * std::fabs(L)) ++nbad;
      L = L2;
    }
  }
  if (bad) *bad = nbad;
  return delta;
}

// One GCD sweep [Alg. 2]: E_best = FindBest(m), sequential updates in rank
// order, then the theta update (R6).  Returns Delta; writes the objective.
double orc_gcd_sweep(void* h, int64_t m, int mode, uint64_t seed, double eps, int max_iter,
                     double* objective_out, int64_t* n_best) {
  Problem& P = *(Problem*)h;
  std::vector<int32_t> I(m), J(m);
  std::vector<double> G(m);
  int64_t n = orc_find_best(h, m, mode, seed, eps, max_iter, I.data(), J.data(), G.data(), nullptr);
  // Only the positive gains among the best m are applied: a zero-gain pair
  // leaves W unchanged when it is picked, and the paper's arbitrary tie
  // breaking is read as picking none of the zero-gain ties.  (Ranked by the
  // gradient distance, the list is not ordered by gain: all of it is applied.)
  if (P.dist == 0) {
    int64_t pos = 0;
    while (pos < n && G[pos] > 0.0) ++pos;
    n = pos;
  }
  double delta = orc_apply_updates(h, n, I.data(), J.data(), 0, nullptr);
  theta_update(P);
  if (objective_out) *objective_out = objective(P);
  if (n_best) *n_best = n;
  return delta;
}

// One CD sweep [Alg. 1]: every coordinate once, then theta.  The paper leaves
// the visiting order open.  order 0: index order (i, then j).  order 1:
// round-robin rounds (the circle method): with n = N rounded up to even and
// node n - 1 a phantom when N is odd, round r = 0..n-2 pairs r with n - 1 and
// (r + k) mod (n - 1) with (r - k) mod (n - 1) for k = 1..n/2 - 1, in that
// order of k; every unordered pair appears in exactly one round, and a
// round's pairs share no node.  Symmetric models update the pair (min, max);
// the kinetic model updates both ordered couplings of the pair, (a <- b) then
// (b <- a), with a the first node listed above.
double orc_cd_sweep_order(void* h, int order) {
  Problem& P = *(Problem*)h;
  double delta = 0.0;
  auto visit = [&](int i, int j) {
    double g, w;
    pair_gain(P, i, j, &g, &w);
    delta += std::fabs(w - P.w(i, j));
    set_w(P, i, j, w);
  };
  if (order == 0) {
    for (int i = 0; i < P.N; ++i)
      for (int j = 0; j < P.N; ++j) {
        if (i == j || (P.model != KINETIC && j < i)) continue;
        visit(i, j);
      }
  } else {
    const int64_t n = P.N + (P.N & 1);
    for (int64_t r = 0; r + 1 < n; ++r)
      for (int64_t k = 0; k < n / 2; ++k) {
        int64_t a, b;
        if (k == 0) { a = r; b = n - 1; }
        else { a = (r + k) % (n - 1); b = (r - k + (n - 1)) % (n - 1); }
        if (a >= P.N || b >= P.N) continue;   // the phantom node
        if (P.model == KINETIC) {
          visit((int)a, (int)b);
          visit((int)b, (int)a);
        } else {
          visit((int)std::min(a, b), (int)std::max(a, b));
        }
      }
  }
  theta_update(P);
  return delta;
}

double orc_cd_sweep(void* h) { return orc_cd_sweep_order(h, 0); }

// Search distance: 0 the exact gain, 1 the absolute gradient (pair_grad).
void orc_set_dist(void* h, int dist) { ((Problem*)h)->dist = dist; }

// Absolute gradients of pairs (pair_grad), whatever the search distance.
void orc_grad_pairs(void* h, int64_t n, const int32_t* I, const int32_t* J, double* out) {
  Problem& P = *(Problem*)h;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) out[p] = pair_grad(P, I[p], J[p]);
}

// exported numerics for the pin tests
double orc_lcosh(double x) { return lcosh(x); }
double orc_dlcosh(double a, double d) { return dlcosh(a, d); }
uint64_t orc_ctr(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) { return ctr(seed, stream, a, b); }

}  // extern "C"
