/*
 * rec.h -- C ABI of the MI355X (gfx950) library for greedy coordinate descent
 * (GCD) network reconstruction, after T. P. Peixoto, "Scalable network
 * reconstruction in subquadratic time", arXiv 2401.01404.
 *
 * Problem [Sec. 2]: data X, an N x M matrix of M samples (or a Markov time
 * series) of N nodes; unknown weights W (N x N, symmetric for the Ising and
 * Gaussian models, directed for the kinetic Ising model) and node parameters
 * theta; objective pi(W) = log pseudolikelihood [App. A] minus an L1
 * (Laplace) penalty lambda * sum |W_ij| [App. A], maximised by GCD
 * [Alg. 2] whose candidate search is FindBest [Alg. 3] over NNDescent
 * [Alg. 4].  The score of a pair is the gain
 *     gain(i,j) = max_w pi(W with W_ij = w) - pi(W)  >= 0,
 * the negative of the paper's distance d(i,j) = -max_{W_ij} pi(W) up to the
 * constant pi(W) [Alg. 2, function D].
 *
 * Conventions shared by every call:
 *   - Every call returns rec_status; nothing throws across the ABI.
 *   - Pointers named *_dev are device pointers (HIP global memory); *_host are
 *     host pointers.  A call with a *_host output synchronises the context's
 *     stream before it returns; all other work is queued on that stream.
 *   - The caller owns X, the workspace and every output buffer; they must stay
 *     valid until the queued work has finished.  The library allocates no
 *     device memory: all of its state lives in the caller's workspace.
 *   - Node indices are int32 in [0, N).  Symmetric models treat (i,j) and
 *     (j,i) as one coordinate; the kinetic model's pair (i,j) is the ordered
 *     coupling W_ij of source j on target i.
 *   - A context is not thread safe; calls on one context must be serialised.
 *   - Invalid arguments return REC_E_INVAL and change nothing.  A failure in
 *     the middle of a sweep leaves the context in REC_E_STATE until
 *     rec_set_model() restores a consistent model.  rec_last_error() gives a
 *     per-context message for the last failure.
 */
#ifndef REC_H
#define REC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rec_ctx rec_ctx;

typedef enum {
  REC_OK = 0,
  REC_E_INVAL = -1,     /* bad argument (null pointer, index out of range, size) */
  REC_E_NOMEM = -2,     /* workspace too small for the request                   */
  REC_E_HIP = -3,       /* a HIP runtime call failed                             */
  REC_E_NUMERIC = -4,   /* non-finite value in data or result                    */
  REC_E_STATE = -5      /* context poisoned by an earlier failure                */
} rec_status;

/* Generative model of the data [App. A; Sec. 2 Markov product form]. */
typedef enum {
  REC_ISING = 0,        /* +-1 samples, symmetric W, pseudolikelihood prod_i e^{x_i h_i}/2cosh h_i */
  REC_GAUSS = 1,        /* real samples, symmetric W, Gaussian pseudolikelihood, theta_i = 1/sqrt(W_ii) */
  REC_KINETIC = 2       /* +-1 time series x_0..x_M, directed W, P(x_t | x_{t-1}) */
} rec_model;

typedef enum { REC_FP64 = 0, REC_FP32 = 1 } rec_prec;   /* arithmetic of fields and scores */
typedef enum { REC_X_INT8 = 0, REC_X_FP32 = 1 } rec_xtype;

typedef enum {
  REC_SEARCH_NNDESCENT = 0,   /* FindBest [Alg. 3] over NNDescent [Alg. 4]      */
  REC_SEARCH_EXHAUSTIVE = 1,  /* all pairs scored exactly, best m kept         */
  REC_SEARCH_SURROGATE = 2,   /* learned proposal ahead of NNDescent            */
  REC_SEARCH_EXACT_KNN = 3,   /* FindBest [Alg. 3] over exhaustive KNN lists    */
  REC_SEARCH_SCREEN = 4,      /* every pair screened at once by an MFMA
                                 contraction of samples with residuals (the
                                 gradient at the current state, Gaussian: BF16,
                                 Ising/kinetic: int8) under proven bounds on
                                 each pair's gain; survivors and current
                                 couplings rescored exactly.  Returns the
                                 exhaustive search's positive-gain top m
                                 (kinetic: ordered pairs).                     */
  REC_SEARCH_GRADIENT = 5     /* FindBest [Alg. 3] over NNDescent [Alg. 4]
                                 with the gradient as distance [Appendix,
                                 "Gradient as distance"]: every search score
                                 is the absolute gradient of rec_grad_pairs,
                                 and E_best is the best m by that score (each
                                 update still takes the exact coordinate
                                 maximum).  The gains written by
                                 rec_find_best_candidates are those scores. */
} rec_search;

typedef struct {
  int32_t model;          /* rec_model                                                  */
  int32_t xtype;          /* rec_xtype: REC_X_INT8 (+-1) for Ising/kinetic, REC_X_FP32 for Gauss */
  int32_t prec;           /* rec_prec                                                   */
  int32_t knn_k_override; /* 0: k = ceil(4m/|S|) [Alg. 3]; >0: fixed k at every level   */
  int64_t N;              /* nodes, 2 <= N <= 2^20                                       */
  int64_t M;              /* samples (kinetic: transitions; X then has M+1 columns)      */
  int64_t ldx;            /* row stride of X in elements (node-major: X[i*ldx + m])      */
  double lambda;          /* L1 penalty, >= 0, in units of the summed log-likelihood     */
  double kappa;           /* greediness: m = round-half-up(kappa * N), at least 1 [Alg. 2] */
  double nnd_eps;         /* NNDescent stop: changes / (k |S|) < nnd_eps [Alg. 4]        */
  int32_t nnd_max_iter;   /* 0: 2 ceil(log_{2k} |S|) + 10                                */
  int32_t reserved0;
  uint64_t seed;          /* seed of the NNDescent initial lists and in-neighbour caps  */
  int64_t max_nnz;        /* capacity for nonzero W entries (0: 64 * N)                  */
  int32_t log2_cache;     /* score cache slots = 2^log2_cache, <= 30 (0: chosen from N)  */
  int32_t reserved1;
} rec_config;

typedef struct {
  double objective;       /* log pi(W) after the sweep (FP64 sum)                    */
  double delta;           /* sum |W'_ij - W_ij| over the sweep's updates [Alg. 2]    */
  int64_t accepted;       /* pairs of E_best whose weight changed                     */
  int64_t n_best;         /* |E_best|                                                 */
  int64_t pair_evals;     /* exact pair scores computed (cache hits not counted)      */
  int64_t nnd_iters;      /* NNDescent iterations summed over FindBest levels         */
  int64_t levels;         /* FindBest recursion levels                                */
  int64_t rounds;         /* node-disjoint update rounds (kinetic: longest row chain) */
  double t_search_ms;     /* wall time of FindBest                                     */
  double t_update_ms;     /* wall time of the coordinate updates                       */
  double t_theta_ms;      /* wall time of theta update, field refresh and objective    */
} rec_sweep_stats;

/* Bytes of workspace the library needs for cfg.  Host-only; no device work. */
rec_status rec_workspace_size(const rec_config* cfg, size_t* bytes);

/* Create a context on the current HIP device: the reconstruction problem of
 * [Sec. 2] (N x M data X of M samples, or of a time series [Sec. 2, Markov
 * product form]; unknown W and theta) with the objective of [App. A] (log
 * pseudolikelihood of the chosen model plus the Laplace prior of weight
 * lambda on W).  X_dev: node-major data (int8 +-1 or float32, see cfg->xtype)
 * with row stride cfg->ldx; it is copied into the workspace (padded layout),
 * so X_dev may be freed after the call.
 * ws_dev: at least rec_workspace_size() bytes, 256-byte aligned.
 * stream: the hipStream_t to queue all work on (NULL = default stream).
 * Starts from W = 0 [Alg. 2, initial state] with theta at the W = 0 optimum of
 * every node's conditional (theta is fitted alongside W [App. A]).  Also looks
 * up, once per device, the address of the static scratch used by
 * rec_score_pairs_noalloc.  Synchronises the stream.  REC_E_NUMERIC if X holds
 * a value other than +-1 (int8 models) or a non-finite value (float32). */
rec_status rec_create(const rec_config* cfg, const void* X_dev, void* ws_dev, size_t ws_bytes,
                      void* stream, rec_ctx** out);

/* Release the context's host-side state.  The workspace and X belong to the
 * caller and are not touched; queued work must have finished. */
rec_status rec_destroy(rec_ctx* ctx);

/* Exact scores of P pairs at the current state [Alg. 2, function D]:
 * gain_dev[p] = max_w pi(W_{i_p j_p} <- w) - pi(W), wopt_dev[p] = its argmax.
 * i_dev, j_dev: P int32 indices; gain_dev, wopt_dev: P doubles (wopt_dev may
 * be NULL).  FP64 mode computes everything in double; FP32 mode computes the
 * per-sample terms in float with FP64 sums.  Synchronises the stream at the end
 * to report invalid pairs (REC_E_INVAL: any index outside [0,N) or i == j;
 * such pairs get gain NaN). */
rec_status rec_score_pairs(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                           double* gain_dev, double* wopt_dev);

/* rec_score_pairs without any workspace scratch, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and the same results bit for bit, but
 * the per-call scratch (the kink screen's queue and counter, the error flags)
 * is a file-scope static device array of 4 MiB + 256 bytes that each GPU the
 * library runs on holds until the process ends; its address is looked up once
 * per device by rec_create().  At most 2^20 pairs per call (REC_E_INVAL
 * beyond).  Clears what must start at zero with a kernel (no memset), queues
 * no timing events and counts no work.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (several streams or threads)
 * race and must be serialised by the caller.  Arguments, layout, ownership
 * and errors as rec_score_pairs; also synchronises the stream at the end. */
rec_status rec_score_pairs_noalloc(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                                   double* gain_dev, double* wopt_dev);

/* Gradient distance of P pairs at the current state [Appendix, "Gradient as
 * distance"]: dist_dev[p] = |dpi/dW_ij| taken as a central difference at the
 * L1 kink, i.e. |F'(w0) - lambda sign(w0)| for a current coupling w0 != 0 and
 * |F'(0)| for w0 = 0, with F the objective without the penalty, restricted to
 * W_ij.  F' is one pass over the samples: for row a's conditional
 * sum_m x_b,m (y_a,m - tanh h_a,m) (Ising, kinetic) or -sum_m r_a,m x_b,m
 * (Gaussian), summed over both conditionals for the symmetric models; kinetic
 * pairs are ordered (i <- j).  i_dev, j_dev: P int32 indices; dist_dev: P
 * doubles (FP32 mode rounds each to float).  Synchronises the stream;
 * REC_E_INVAL for an index outside [0,N) or i == j (that entry NaN). */
rec_status rec_grad_pairs(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                          double* dist_dev);

/* The m best pairs at the current state [Alg. 3 when s is a FindBest search].
 * Writes up to m pairs best first (gain desc, then min(i,j), max(i,j);
 * kinetic: gain desc, i, j) into i_dev/j_dev/gain_dev (capacity m each) and
 * their count into *n_out_host.  For the kinetic model FindBest runs over
 * unordered pairs scored by max(gain(i <- j), gain(j <- i)), and the m best
 * directed pairs are taken from both directions of the m pairs it finds.
 * stats_host may be NULL; if given, its search fields are filled (pair_evals
 * counts directed scores for the kinetic model).  Synchronises. */
rec_status rec_find_best_candidates(rec_ctx* ctx, int64_t m, int32_t search, int32_t* i_dev, int32_t* j_dev,
                         double* gain_dev, int64_t* n_out_host, rec_sweep_stats* stats_host);

/* Node count N_t of every recursion level t of the last FindBest search
 * [Alg. 3] on this context (the set S of level t; N_0 = N): *levels_host gets
 * the number of levels (0 after an exhaustive or screened search, which has
 * none), level_n_host its first min(cap, levels) counts.  Host-only; no
 * device work.  For comparing the recursion with Sec. 3's prediction
 * s_{t+1} = F(ceil(4 kappa / s_t)), s_t = N_t / N, F the tail distribution
 * of the degrees of the pairs found. */
rec_status rec_search_levels(rec_ctx* ctx, int32_t cap, int64_t* level_n_host, int32_t* levels_host);

/* One GCD iteration [Alg. 2]: E_best = FindBest(m = round(kappa N)); every
 * pair of E_best updated to its argmax in rank order (run as node-disjoint
 * rounds, for the kinetic model as one chain per target row, either of which
 * equals the sequential order); then theta refitted for all
 * nodes, fields rebuilt from W and the objective evaluated.  Synchronises. */
rec_status rec_gcd_sweep(rec_ctx* ctx, int32_t search, rec_sweep_stats* stats_host);

/* Apply coordinate updates to the given P pairs in the given order
 * [Alg. 2 loop body]: each W_ij set to its argmax with the current state.
 * Writes Delta = sum |W' - W| to *delta_host.  Synchronises. */
rec_status rec_apply_updates(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                             double* delta_host);

/* One sweep of the coordinate-descent baseline [Alg. 1]: every coordinate
 * W_ij set to its argmax at the current state, each once, then theta refitted
 * for all nodes, the fields rebuilt from W and the objective evaluated, as at
 * the end of rec_gcd_sweep.  The paper leaves the visiting order open; here it
 * is the round-robin (circle method) order: with n = N rounded up to even
 * (node n - 1 a phantom when N is odd), round r = 0..n-2 visits the pairs
 * (r, n - 1) and ((r + k) mod (n - 1), (r - k) mod (n - 1)), k = 1..n/2 - 1;
 * a round's pairs share no node, so each round runs as one parallel launch and
 * gives the sequential result.  Symmetric models update the pair (min, max);
 * the kinetic model both ordered couplings (a <- b), then (b <- a).
 * stats_host (may be NULL): objective, delta = sum |dW|, accepted = changed
 * couplings, n_best = pair_evals = coordinates visited, rounds = n - 1,
 * t_update_ms (the rounds), t_theta_ms.  O(N^2 M) work per sweep.
 * REC_E_NOMEM if the couplings outgrow cfg.max_nnz (the context is then left
 * in REC_E_STATE).  Synchronises. */
rec_status rec_cd_sweep(rec_ctx* ctx, rec_sweep_stats* stats_host);

/* Refit theta for all nodes, rebuild fields from W and return log pi(W)
 * [App. A].  Synchronises. */
rec_status rec_theta_update(rec_ctx* ctx, double* objective_host);

/* log pi(W) at the current state (FP64 sum).  Synchronises. */
rec_status rec_objective(rec_ctx* ctx, double* objective_host);

/* Export the model [Sec. 2: the reconstruction is the pair (W, theta); App. A:
 * theta_i = 1/sqrt(W_ii) for the Gaussian model, the field of node i for the
 * Ising models]: nonzero W entries (symmetric: i < j; kinetic: ei = target,
 * ej = source) into ei/ej/w (capacity cap, sorted by (ei, ej)) and theta
 * (N doubles, may be NULL).  *nnz_host receives the number of nonzero entries
 * (which may exceed cap).  Synchronises. */
rec_status rec_get_model(rec_ctx* ctx, int64_t cap, int32_t* ei_dev, int32_t* ej_dev,
                         double* w_dev, double* theta_dev, int64_t* nnz_host);

/* Replace the model (W entries and theta [Sec. 2; App. A], as rec_get_model
 * writes them; theta_dev NULL keeps theta) and rebuild the local fields from
 * them (h_i = theta_i + sum_j W_ij x_j [App. A]), so that
 * rec_set_model(rec_get_model()) restores the state bit for bit.  For resuming,
 * or for starting from a model computed elsewhere.  Entries must have
 * distinct coordinates with finite weights (REC_E_INVAL; the context is then
 * left in REC_E_STATE); more than cfg.max_nnz entries give REC_E_NOMEM.
 * Clears REC_E_STATE.  Synchronises. */
rec_status rec_set_model(rec_ctx* ctx, int64_t nnz, const int32_t* ei_dev, const int32_t* ej_dev,
                         const double* w_dev, const double* theta_dev);

/* Fields in the working precision, converted to double: h = theta + sum_j W_ij x_j
 * (Gaussian: residual x_i + theta_i^2 sum_j W_ij x_j), N x M row-major. */
rec_status rec_get_fields(rec_ctx* ctx, double* H_dev);

/* KNN lists of FindKNN [Alg. 4] (mode REC_SEARCH_NNDESCENT; REC_SEARCH_GRADIENT
 * for NNDescent under the gradient distance of rec_grad_pairs) or exact KNN
 * (REC_SEARCH_EXACT_KNN) over the node subset S (n sorted indices) at
 * FindBest level `level`: writes n*k neighbour indices and scores, best first
 * per node; *iters_host gets the NNDescent iteration count (kinetic model:
 * under the score max(d(i <- j), d(j <- i))).  Synchronises. */
rec_status rec_knn(rec_ctx* ctx, int64_t n, const int32_t* S_dev, int32_t k, int32_t level,
                   int32_t mode, int32_t* nbr_dev, double* gain_dev, int32_t* iters_host);

/* ---- Learned proposal (not part of the paper) --------------------------
 * A ranking MLP over per-node sketches orders the candidate pairs of the
 * second-neighbour search [Alg. 4] so that only the most promising fraction
 * is scored exactly [Alg. 2, function D]; the exact score judges every pair
 * that enters a list.  Sketch of node i (64 floats): 28 + 28 random +-1
 * projections P(x_i + r_i)/sqrt(M), P(x_i - r_i)/sqrt(M) (r = y - tanh h;
 * Gaussian: the residual; P[d][m] = -1 iff the top bit of SplitMix64
 * ctr(seed, 7, d, m) is set), then mean y, mean t, var t, mean |h|, mean r^2,
 * log(1 + degree), sum |W_i.|, theta_i.  Pair feature: [s_i*s_j, |s_i-s_j|,
 * s_i+s_j] (192) -> 128 -> 128 -> 1 with ReLU; trained on log(1 + gain).
 * Flat parameters (REC_SUR_NPARAM floats): W1[192][128], b1[128],
 * W2[128][128], b2[128], w3[128], b3. */
#define REC_SUR_SKETCH_DIM 64
#define REC_SUR_NPARAM 41345
#define REC_SUR_MAX_BATCH 8192

/* Sketches of every node at the current state into the context (and into
 * S_dev, N x 64 floats, when not NULL).  Synchronises. */
rec_status rec_sketch(rec_ctx* ctx, float* S_dev);

/* Copy the parameters out to get_dev (may be NULL), then replace them by
 * set_dev (may be NULL; resets the Adam state).  Device pointers of
 * REC_SUR_NPARAM floats.  Synchronises. */
rec_status rec_mlp_params(rec_ctx* ctx, float* get_dev, const float* set_dev);

/* MLP scores of P pairs under the context's sketches (BF16 MFMA with FP32
 * accumulation; h1 rounded to bf16 between the layers).  Synchronises. */
rec_status rec_mlp_infer(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                         float* out_dev);

/* FP32 loss mean (out - y)^2 / 2 and its gradient for a batch of
 * 1 <= P <= REC_SUR_MAX_BATCH pairs with targets y_dev (grad_dev: NPARAM
 * floats, may be NULL).  Synchronises. */
rec_status rec_mlp_grad(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                        const float* y_dev, float* grad_dev, double* loss_host);

/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8, bias-corrected) on one batch;
 * *loss_host gets the loss before the last step.  Synchronises. */
rec_status rec_mlp_train(rec_ctx* ctx, int64_t P, const int32_t* i_dev, const int32_t* j_dev,
                         const float* y_dev, int32_t steps, float lr, double* loss_host);

/* The proposal inside FindBest (search REC_SEARCH_SURROGATE, NNDescent
 * underneath).  rho: fraction of each candidate chunk scored exactly (by
 * predicted rank); recall_min: the proposal filters only while its last
 * recall estimate of positive-gain candidates reaches this (else the plain
 * search runs and the network is evaluated in shadow: exact recall); after
 * every such FindBest call the network takes train_steps Adam steps (lr) on
 * the call's exact scores (all positive gains, zeros sampled 1 in
 * 2^zero_log2); 1 in 2^audit_log2 of the filtered-out candidates is scored
 * anyway to estimate the recall.  Defaults: 0.25, 0.99, 50, 1e-3, 4, 6. */
rec_status rec_surrogate_config(rec_ctx* ctx, double rho, double recall_min, int32_t train_steps,
                                float lr, int32_t audit_log2, int32_t zero_log2);

/* After the last REC_SEARCH_SURROGATE call: [0] 1 = plain search with
 * shadow evaluation, 2 = filtered; [1] recall estimate; [2] fraction of
 * candidates scored exactly; [3] positives kept; [4] positives missed
 * (estimated when filtered); [5], [6] training records (positive, zero);
 * [7] training loss; [8] calls so far; [9] rho.  Host array of 10. */
rec_status rec_surrogate_stats(rec_ctx* ctx, double* out_host);

/* Instrumentation (not part of the method): when on, every launch of the
 * pair-score kernel is bracketed by HIP events on the context's stream.
 * rec_kernel_time returns, for the launches since the last call (or since
 * timing was switched on), the summed kernel time in ms, the number of
 * launches and eight work counters (work_host: 8 int64, may be NULL): pairs
 * scored, moment passes, full Newton evaluations, log passes (each pass is
 * one sweep over the M samples of the pair's one or two sides), pair sides
 * settled by the int8 residual screen, j-side rows fetched, i-side row
 * loads, and the algorithmic bytes the kernels read and write (indices,
 * scores and the rows they need, at M samples).  Synchronises; resets the
 * sums. */
rec_status rec_set_timing(rec_ctx* ctx, int32_t on);
rec_status rec_kernel_time(rec_ctx* ctx, double* score_ms_host, int64_t* launches_host,
                           int64_t* work_host);

/* Instrumentation of REC_SEARCH_SCREEN, since the last call (or since
 * rec_set_timing): out_host (9 doubles) = [0] kernel ms of the full
 * contraction passes (event-timed while timing is on), [1] their launches,
 * [2] their algorithmic flops (2 M flops per ordered pair for the kinetic
 * model, per unordered pair and side for the symmetric ones), [3] kernel ms
 * of the sampling passes, [4] their launches, [5] screen calls, [6] pairs
 * decided (every pair of each call: scored exactly or excluded by the
 * bounds), [7] pairs rescored exactly, [8] calls that needed a second
 * collect pass.  Synchronises; resets the sums. */
rec_status rec_screen_time(rec_ctx* ctx, double* out_host);

const char* rec_status_str(rec_status s);
const char* rec_last_error(const rec_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* REC_H */
