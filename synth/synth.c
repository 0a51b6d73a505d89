/*
 * Seeded synthetic workload generators: random graphs, coupling weights and
 * samplers for the Ising, kinetic-Ising and Gaussian models.
 *
 * These produce the data matrix X that both the GPU library and the CPU
 * oracle consume.  Nothing here computes any quantity of the reconstruction
 * method itself (no pseudolikelihood, no score, no search); it only draws
 * samples from the generative models of the paper's Appendix A (Ising and
 * Gaussian) and from the Markov product form of Section 2 (kinetic Ising).
 *
 * Randomness is counter based: every draw is SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to a key built from (seed, stream, a, b), so results do not depend
 * on thread count or loop order.
 *
 * Layout of every data matrix: node-major, element (i, m) at X[i*ldx + m].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- RNG --- */

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* key(seed, stream, a, b): one 64-bit random word per counter tuple */
static inline uint64_t ctr(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(mix64(seed) ^ stream) ^ a) ^ b);
}

/* uniform in [0, 1) with 53 random bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* standard normal by Box-Muller from two counter draws */
static inline double normal01(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  double u1 = u01(ctr(seed, stream, a, 2 * b));
  double u2 = u01(ctr(seed, stream, a, 2 * b + 1));
  return sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
}

uint64_t synth_mix64(uint64_t z) { return mix64(z); }
uint64_t synth_ctr(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  return ctr(seed, stream, a, b);
}

/* Stream ids, fixed so that every workload is reproducible from its seed. */
enum {
  ST_GRAPH = 1, ST_WEIGHT = 2, ST_START = 3, ST_GIBBS = 4, ST_THETA = 9,
  ST_GAUSS = 7, ST_GLAUBER = 8, ST_REGULAR = 10
};

/* ---------------------------------------------------------- graphs ------ */

/*
 * Erdos-Renyi G(N, p) on unordered pairs by geometric skipping (Batagelj and
 * Brandes, "Efficient generation of large random networks", PRE 71, 2005).
 * Writes at most cap edges (v > w) and returns the total count; a count above
 * cap means the arrays were too small (call again with a bigger cap).
 */
int64_t synth_er_undirected(int64_t N, double p, uint64_t seed, int64_t cap,
                            int32_t* ei, int32_t* ej) {
  if (N < 2 || p <= 0.0) return 0;
  double lq = log1p(-p);
  int64_t v = 1, w = -1, count = 0, draw = 0;
  while (v < N) {
    double r = u01(ctr(seed, ST_GRAPH, 0, (uint64_t)draw++));
    w = w + 1 + (int64_t)floor(log1p(-r) / lq);
    while (w >= v && v < N) { w -= v; v++; }
    if (v < N) {
      if (count < cap) { ei[count] = (int32_t)w; ej[count] = (int32_t)v; }
      count++;
    }
  }
  return count;
}

/*
 * Directed G(N, p) over ordered pairs (dst, src), dst != src, same skipping
 * over the N*(N-1) linear index.  An edge src -> dst means that node src
 * drives node dst, i.e. coupling W[dst][src] is nonzero.
 */
int64_t synth_er_directed(int64_t N, double p, uint64_t seed, int64_t cap,
                          int32_t* dst, int32_t* src) {
  if (N < 2 || p <= 0.0) return 0;
  double lq = log1p(-p);
  int64_t total = N * (N - 1), idx = -1, count = 0, draw = 0;
  for (;;) {
    double r = u01(ctr(seed, ST_GRAPH, 1, (uint64_t)draw++));
    idx = idx + 1 + (int64_t)floor(log1p(-r) / lq);
    if (idx >= total) break;
    int64_t row = idx / (N - 1), c = idx % (N - 1);
    int64_t col = c < row ? c : c + 1;
    if (count < cap) { dst[count] = (int32_t)row; src[count] = (int32_t)col; }
    count++;
  }
  return count;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y);
}

/*
 * Random d-regular simple graph by the configuration model: shuffle N*d
 * stubs, pair them in order, and redraw the whole pairing while it holds a
 * loop or a repeated edge.  Returns N*d/2 edges, or -1 if N*d is odd or no
 * simple pairing was found in max_tries.
 */
int64_t synth_regular(int64_t N, int d, uint64_t seed, int max_tries,
                      int32_t* ei, int32_t* ej) {
  int64_t S = N * (int64_t)d;
  if (S % 2) return -1;
  int32_t* stub = (int32_t*)malloc(sizeof(int32_t) * S);
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (S / 2));
  int64_t result = -1;
  for (int t = 0; t < max_tries && result < 0; t++) {
    for (int64_t s = 0; s < S; s++) stub[s] = (int32_t)(s / d);
    for (int64_t s = S - 1; s > 0; s--) {   /* Fisher-Yates */
      uint64_t r = ctr(seed, ST_REGULAR, (uint64_t)t, (uint64_t)s);
      int64_t k = (int64_t)(((unsigned __int128)r * (uint64_t)(s + 1)) >> 64);
      int32_t tmp = stub[s]; stub[s] = stub[k]; stub[k] = tmp;
    }
    int ok = 1;
    for (int64_t e = 0; e < S / 2; e++) {
      int32_t a = stub[2 * e], b = stub[2 * e + 1];
      if (a == b) { ok = 0; break; }
      uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
      key[e] = (lo << 32) | hi;
    }
    if (!ok) continue;
    qsort(key, S / 2, sizeof(uint64_t), cmp_u64);
    for (int64_t e = 1; e < S / 2; e++)
      if (key[e] == key[e - 1]) { ok = 0; break; }
    if (!ok) continue;
    for (int64_t e = 0; e < S / 2; e++) {
      ei[e] = (int32_t)(key[e] >> 32); ej[e] = (int32_t)(key[e] & 0xffffffffu);
    }
    result = S / 2;
  }
  free(stub); free(key);
  return result;
}

/* ---------------------------------------------------------- weights ----- */

void synth_normal(int64_t n, double mu, double sigma, uint64_t seed, uint64_t stream,
                  double* out) {
  for (int64_t k = 0; k < n; k++) out[k] = mu + sigma * normal01(seed, stream, 0, (uint64_t)k);
}

void synth_uniform(int64_t n, double lo, double hi, uint64_t seed, uint64_t stream,
                   double* out) {
  for (int64_t k = 0; k < n; k++) out[k] = lo + (hi - lo) * u01(ctr(seed, stream, 1, (uint64_t)k));
}

/* -------------------------------------------------- adjacency helper ---- */

typedef struct { int64_t* off; int32_t* nb; double* w; } csr_t;

/* symmetric CSR from undirected (ei, ej, w) */
static csr_t csr_sym(int64_t N, int64_t nnz, const int32_t* ei, const int32_t* ej,
                     const double* w) {
  csr_t g;
  g.off = (int64_t*)calloc(N + 1, sizeof(int64_t));
  g.nb = (int32_t*)malloc(sizeof(int32_t) * (2 * nnz + 1));
  g.w = (double*)malloc(sizeof(double) * (2 * nnz + 1));
  for (int64_t e = 0; e < nnz; e++) { g.off[ei[e] + 1]++; g.off[ej[e] + 1]++; }
  for (int64_t i = 0; i < N; i++) g.off[i + 1] += g.off[i];
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  memcpy(cur, g.off, sizeof(int64_t) * (N + 1));
  for (int64_t e = 0; e < nnz; e++) {
    int64_t a = cur[ei[e]]++, b = cur[ej[e]]++;
    g.nb[a] = ej[e]; g.w[a] = w[e];
    g.nb[b] = ei[e]; g.w[b] = w[e];
  }
  free(cur);
  return g;
}

/* directed in-adjacency: row dst lists its sources */
static csr_t csr_in(int64_t N, int64_t nnz, const int32_t* dst, const int32_t* src,
                    const double* w) {
  csr_t g;
  g.off = (int64_t*)calloc(N + 1, sizeof(int64_t));
  g.nb = (int32_t*)malloc(sizeof(int32_t) * (nnz + 1));
  g.w = (double*)malloc(sizeof(double) * (nnz + 1));
  for (int64_t e = 0; e < nnz; e++) g.off[dst[e] + 1]++;
  for (int64_t i = 0; i < N; i++) g.off[i + 1] += g.off[i];
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  memcpy(cur, g.off, sizeof(int64_t) * (N + 1));
  for (int64_t e = 0; e < nnz; e++) {
    int64_t a = cur[dst[e]]++;
    g.nb[a] = src[e]; g.w[a] = w[e];
  }
  free(cur);
  return g;
}

static void csr_free(csr_t g) { free(g.off); free(g.nb); free(g.w); }

/* ---------------------------------------------------------- samplers ---- */

/*
 * Equilibrium Ising samples by single-site heat-bath Gibbs sampling with a
 * systematic scan i = 0..N-1.  Start: uniform +-1.  Sample m is the state
 * after burn + thin*m full sweeps (m = 0..M-1).  Model (Appendix A):
 * P(x) ~ exp(sum_{i<j} W_ij x_i x_j + sum_i theta_i x_i), so the conditional
 * of x_i is P(x_i = +1 | rest) = 1 / (1 + exp(-2 h_i)) with
 * h_i = theta_i + sum_j W_ij x_j.
 */
int synth_gibbs(int64_t N, int64_t M, int64_t nnz, const int32_t* ei, const int32_t* ej,
                const double* w, const double* theta, int64_t burn, int64_t thin,
                uint64_t seed, int8_t* X, int64_t ldx) {
  if (N <= 0 || M <= 0 || ldx < M || burn < 1 || thin < 1) return -1;
  csr_t g = csr_sym(N, nnz, ei, ej, w);
  int8_t* x = (int8_t*)malloc(N);
  for (int64_t i = 0; i < N; i++) x[i] = (ctr(seed, ST_START, 0, (uint64_t)i) >> 63) ? 1 : -1;
  int64_t next = burn, m = 0;
  for (int64_t s = 1; m < M; s++) {
    for (int64_t i = 0; i < N; i++) {
      double h = theta ? theta[i] : 0.0;
      for (int64_t a = g.off[i]; a < g.off[i + 1]; a++) h += g.w[a] * x[g.nb[a]];
      double p = 1.0 / (1.0 + exp(-2.0 * h));
      double u = u01(ctr(seed, ST_GIBBS, (uint64_t)s, (uint64_t)i));
      x[i] = u < p ? 1 : -1;
    }
    if (s == next && m < M) {
      for (int64_t i = 0; i < N; i++) X[i * ldx + m] = x[i];
      m++;
      next += thin;
    }
  }
  free(x);
  csr_free(g);
  return 0;
}

/*
 * Kinetic Ising time series by parallel Glauber dynamics: from a uniform
 * +-1 state x_0, every node at once draws
 * P(x_{i,t+1} = +1 | x_t) = 1 / (1 + exp(-2 h_{i,t})),
 * h_{i,t} = theta_i + sum_j W_ij x_{j,t}.  X gets T+1 columns (t = 0..T).
 * Edges are (dst, src) with weight w: W[dst][src] = w.
 */
int synth_glauber(int64_t N, int64_t T, int64_t nnz, const int32_t* dst, const int32_t* src,
                  const double* w, const double* theta, uint64_t seed, int8_t* X, int64_t ldx) {
  if (N <= 0 || T < 1 || ldx < T + 1) return -1;
  csr_t g = csr_in(N, nnz, dst, src, w);
  for (int64_t i = 0; i < N; i++)
    X[i * ldx + 0] = (ctr(seed, ST_START, 1, (uint64_t)i) >> 63) ? 1 : -1;
  for (int64_t t = 0; t < T; t++) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
      double h = theta ? theta[i] : 0.0;
      for (int64_t a = g.off[i]; a < g.off[i + 1]; a++) h += g.w[a] * X[(int64_t)g.nb[a] * ldx + t];
      double p = 1.0 / (1.0 + exp(-2.0 * h));
      double u = u01(ctr(seed, ST_GLAUBER, (uint64_t)t, (uint64_t)i));
      X[i * ldx + t + 1] = u < p ? 1 : -1;
    }
  }
  csr_free(g);
  return 0;
}

/*
 * Zero-mean Gaussian samples x ~ N(0, Theta^{-1}) for a sparse precision
 * matrix Theta given by its off-diagonal entries (ei < ej, value off) and
 * the diagonal Theta_ii = sum_j |Theta_ij| / (1 - eps)^2 (1 for isolated
 * nodes), the recipe of the paper's synthetic Gaussian data (Section 4).
 *
 * Exact sampler: Theta = B^T B with one row sqrt|Theta_ij| (e_i + sgn e_j)
 * per edge and one row sqrt(Theta_ii - sum_j |Theta_ij|) e_i per node, so
 * x = Theta^{-1} B^T z with z ~ N(0, I) has covariance Theta^{-1}.  The
 * solve is Jacobi-preconditioned conjugate gradients in FP64 to relative
 * residual tol.  Returns the largest CG iteration count, or -1 on failure.
 */
int synth_gauss(int64_t N, int64_t M, int64_t nnz, const int32_t* ei, const int32_t* ej,
                const double* off, double eps, uint64_t seed, double tol, int64_t max_iter,
                float* X, int64_t ldx, double* diag_out) {
  if (N <= 0 || M <= 0 || ldx < M) return -1;
  csr_t g = csr_sym(N, nnz, ei, ej, off);
  double* diag = (double*)malloc(sizeof(double) * N);
  double* resid = (double*)malloc(sizeof(double) * N);
  for (int64_t i = 0; i < N; i++) {
    double s = 0.0;
    for (int64_t a = g.off[i]; a < g.off[i + 1]; a++) s += fabs(g.w[a]);
    diag[i] = s > 0.0 ? s / ((1.0 - eps) * (1.0 - eps)) : 1.0;
    resid[i] = diag[i] - s;
    if (diag_out) diag_out[i] = diag[i];
  }
  int worst = 0;
#pragma omp parallel
  {
    double* b = (double*)malloc(sizeof(double) * N);
    double* x = (double*)malloc(sizeof(double) * N);
    double* r = (double*)malloc(sizeof(double) * N);
    double* z = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    int local_worst = 0;
#pragma omp for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; m++) {
      /* b = B^T z */
      for (int64_t i = 0; i < N; i++) b[i] = sqrt(resid[i]) * normal01(seed, ST_GAUSS, (uint64_t)m, (uint64_t)i);
      for (int64_t e = 0; e < nnz; e++) {
        double zz = normal01(seed, ST_GAUSS, (uint64_t)m, (uint64_t)(N + e));
        double a = sqrt(fabs(off[e]));
        double sg = off[e] >= 0.0 ? 1.0 : -1.0;
        b[ei[e]] += a * zz;
        b[ej[e]] += sg * a * zz;
      }
      double bnorm = 0.0;
      for (int64_t i = 0; i < N; i++) { x[i] = 0.0; r[i] = b[i]; bnorm += b[i] * b[i]; }
      bnorm = sqrt(bnorm);
      double rz = 0.0;
      for (int64_t i = 0; i < N; i++) { z[i] = r[i] / diag[i]; p[i] = z[i]; rz += r[i] * z[i]; }
      int it = 0;
      for (; it < max_iter; it++) {
        double rn = 0.0;
        for (int64_t i = 0; i < N; i++) rn += r[i] * r[i];
        if (sqrt(rn) <= tol * bnorm) break;
        double pq = 0.0;
        for (int64_t i = 0; i < N; i++) {
          double s = diag[i] * p[i];
          for (int64_t a = g.off[i]; a < g.off[i + 1]; a++) s += g.w[a] * p[g.nb[a]];
          q[i] = s;
          pq += p[i] * s;
        }
        double alpha = rz / pq;
        for (int64_t i = 0; i < N; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rz2 = 0.0;
        for (int64_t i = 0; i < N; i++) { z[i] = r[i] / diag[i]; rz2 += r[i] * z[i]; }
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < N; i++) p[i] = z[i] + beta * p[i];
      }
      if (it >= max_iter) local_worst = -1000000000;
      else if (it > local_worst && local_worst >= 0) local_worst = it;
      for (int64_t i = 0; i < N; i++) X[i * ldx + m] = (float)x[i];
    }
#pragma omp critical
    {
      if (local_worst < 0 || worst < 0) worst = -1;
      else if (local_worst > worst) worst = local_worst;
    }
    free(b); free(x); free(r); free(z); free(p); free(q);
  }
  free(diag); free(resid);
  csr_free(g);
  return worst;
}
