/*
 * ns.h -- C ABI of libns.so, an MI355X (gfx950) implementation of the batched
 * nested sampler of "Fast and efficient nested sampling with BEST"
 * (arXiv 2608.28514).
 *
 * The problem (Sec. 1, Eq. (1)): compute the evidence Z = int_0^1 L(X) dX of a
 * likelihood L under a uniform prior on a box [lo, hi], by keeping N live
 * points and repeatedly replacing the worst ones with points of higher
 * likelihood.  One call of ns_step_batch(m) replaces m live points at once
 * (Sec. 3): the m worst are selected by sorting (Algorithm 1), m slice-sampling
 * chains run under the hard constraints L > L_W[j] (Sec. 2.2) with directions
 * whitened by the covariance of the seed's k-means cluster (Sec. 2.1), and the
 * batch is corrected by batch sorting (Algorithm 1) or the history correction
 * (Algorithm 2).  Dead points enter a single-point evidence integration in FP64.
 *
 * Conventions common to every call:
 *  - Every call returns ns_status; a negative value is an error and leaves the
 *    context as it was; ns_last_error(ctx) describes it until the next call.
 *  - Host pointers (const double* lo, likelihood parameters, ...) are read
 *    during the call and copied; the caller keeps ownership.
 *  - Device pointers (arguments named d_*) must point to device memory of the
 *    current HIP device, sized as stated; the library never frees them.
 *  - All device work of a context runs on one HIP stream: the one given to
 *    ns_init, or the default (null) stream when NULL.  Only ns_logZ, ns_sync
 *    and the ns_get_* / ns_*stats getters synchronise that stream.
 *  - Points are stored in unit-cube coordinates u in [0,1]^d, theta = lo +
 *    (hi - lo) u.  Arrays of points are row major: point k occupies
 *    [k*d, (k+1)*d).
 *  - A context is not thread safe; distinct contexts are independent.
 *  - Limits: 1 <= d <= 32, 2 <= N <= 8192, 1 <= m <= min(N-1, 1024),
 *    tree_depth <= 6, hist_cap in [2, 64], lo < hi elementwise.
 */
#ifndef NS_H
#define NS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx; /* opaque; created by ns_init, owned by the library */

typedef enum {
  NS_OK = 0,
  NS_DONE = 1,        /* the stopping rule holds; further steps are no-ops        */
  NS_EINVAL = -1,     /* invalid argument                                         */
  NS_ENOMEM = -2,     /* device or host allocation failed                         */
  NS_EDEVICE = -3,    /* a HIP call failed                                        */
  NS_ESTATE = -4,     /* call not valid in the context's state                    */
  NS_ENUMERIC = -5    /* non-finite value where none is allowed                   */
} ns_status;

/* NS_BF16: bfloat16 MFMA operands, FP32 accumulation.  NS_BF16X3: the same
 * MFMA with each activation split into three bfloat16 terms (hi + mid + lo),
 * which keeps ~24 significant bits of the activations. */
typedef enum { NS_FP64 = 0, NS_FP32 = 1, NS_BF16 = 2, NS_BF16X3 = 3 } ns_prec;

/* Batch corrections, Sec. 3 and Sec. 3.2 (i)-(v). */
typedef enum {
  NS_CORR_NONE = 0,           /* naive: the m worst die, chain j replaces W[j]            */
  NS_CORR_BEST_OF_WORST = 1,  /* every chain uses the batch-best worst L_W[m-1]           */
  NS_CORR_SORT = 2,           /* Algorithm 1: sort W u N, worst m die                     */
  NS_CORR_HISTORY = 3         /* Algorithm 2: Algorithm 1 + history_iters relaxations     */
} ns_corr;

/* Likelihood families (vectorised on the device, except NS_LIK_CALLBACK). */
typedef enum {
  NS_LIK_MIXTURE = 0,    /* log sum_k exp(logw_k - q_k/2), q_k diagonal Mahalanobis:
                            Gaussians, Eq. (2), Eq. (3), Eq. (5) and Gaussian mixtures   */
  NS_LIK_ROSENBROCK = 1, /* -sum_i [b (x_{i+1} - x_i^2)^2 + (a - x_i)^2], Eq. (6)      */
  NS_LIK_SHELL = 2,      /* -((|x| - r0)/w)^2 / 2, Eq. (4)                              */
  NS_LIK_MLP = 3,        /* emulator: tanh MLP, linear output, diagonal chi^2 (Sec. 5)  */
  NS_LIK_CALLBACK = 4    /* any likelihood, evaluated on the host by a user function   */
} ns_lik_kind;

/* Host likelihood for NS_LIK_CALLBACK: logL[k] = log L(theta_k) for the n
 * points theta (n x d, row major, parameter space theta = lo + (hi - lo) u,
 * all inside the prior box), FP64.  Both arrays are host memory owned by the
 * library, valid during the call.  Return 0 on success; any other value stops
 * the step with NS_EINVAL.  NaN results count as -inf and are counted in
 * ns_stats_t.nan_logL; -inf is a valid value (zero likelihood).  The sampler
 * calls it from the thread that calls ns_init / ns_step_batch / ns_run, once
 * per batched round with that round's proposals (the rounds driver is used;
 * with stepout_spec = shrink_spec = 1 every point passed is one counted
 * likelihood evaluation), and synchronises its stream around each call. */
typedef int (*ns_lik_callback)(void* user, const double* theta, int64_t n, int d, double* logL);

typedef struct {
  ns_lik_kind kind;
  ns_prec prec;            /* arithmetic of the likelihood: FP64 or FP32 for analytic
                              families; FP32, BF16 or BF16X3 for MLP (the first layer
                              always runs in FP32 so theta is never rounded)          */
  /* NS_LIK_MIXTURE: n_comp components; logw[K], mu[K*d], ivar[K*d] (host)             */
  int n_comp;
  const double* logw;
  const double* mu;
  const double* ivar;
  /* NS_LIK_ROSENBROCK */
  double ros_a, ros_b;
  /* NS_LIK_SHELL */
  double shell_r0, shell_w;
  /* NS_LIK_MLP: n_layers weight matrices; widths[n_layers+1] with widths[0] == d;
     weights = concatenated row-major W_l (widths[l] x widths[l+1]); biases
     concatenated; data[widths[n_layers]] and sigma[widths[n_layers]] > 0.          */
  int n_layers;
  const int* widths;
  const double* weights;
  const double* biases;
  const double* data;
  const double* sigma;
  /* NS_LIK_CALLBACK: the function and its user pointer (prec must be NS_FP64);
     kept, not copied: both must stay valid while the context lives          */
  ns_lik_callback callback;
  void* callback_user;
} ns_likelihood;

typedef struct {
  int slice_steps_per_dim; /* n: n*d slice iterations per chain (Sec. 2.2); default 5   */
  double step_width;       /* bracket width w in units of the whitened direction; 1.0   */
  int max_stepout;         /* stepping-out cap per side; 64                             */
  int max_shrink;          /* shrink cap; 64                                            */
  int tree_depth;          /* D: at most 2^D clusters (Sec. 2.1); 0 = one cluster       */
  double split_vol_frac;   /* p: children kept if their volume is < (1-p) x parent; 0.3 */
  int min_cluster_pts;     /* n_min: both children need more points; 0 = 2(d+1)        */
  int recluster_every;     /* recluster after this many deaths (Sec. 2.1); 100          */
  int kmeans_iters;        /* Lloyd iteration cap; 20                                   */
  ns_corr correction;      /* default NS_CORR_HISTORY                                   */
  int history_iters;       /* K of Algorithm 2; default 1 (Sec. 3.1)                    */
  int hist_cap;            /* T: stored shrink proposals of the last iteration; 32      */
  ns_prec state_prec;      /* sampler state precision: FP64 or FP32                     */
  double stop_frac;        /* stop when X_i max(L_live) < stop_frac Z_i; 1e-3           */
  double eig_floor;        /* covariance eigenvalue floor, relative to lambda_max; 1e-8 */
  uint64_t seed;           /* Philox4x32-10 key                                         */
  int batch_rounds;        /* 1: evaluate proposals in batched rounds (always the case
                              for NS_LIK_MLP); 0: analytic families run one fused
                              kernel per step                                           */
  int stepout_spec;        /* batched rounds: stepping-out offsets per side per round; 4 */
  int shrink_spec;         /* batched rounds: shrink proposals per round; 8             */
  int fused_chains;        /* network likelihoods: 1 (default) runs a step's chains in
                              one persistent launch whose workgroups evaluate their own
                              rows through the network (FP32 state, split-bfloat16 or
                              FP32 layers, stepout_spec <= 4, shrink_spec <= 8, hidden
                              widths 256 or 512, output 256, 512 or 1024; otherwise,
                              and with the learned screen, the batched-rounds driver);
                              0: always the batched-rounds driver (the same results;
                              with FP32 layers the same to FP32 rounding)           */
  int wait_limit;          /* polls a device-side grid barrier (the one-launch split of
                              a large tree root) makes before it gives up; 0 (default):
                              2^24.  A wait that gives up stops the run, and the next
                              call that synchronises returns NS_EDEVICE              */
} ns_config;

typedef struct {
  int64_t steps;           /* steps that did work                                       */
  int64_t dead;            /* dead rows (live-point updates)                            */
  int64_t evals;           /* true likelihood evaluations of in-box points (incl. init) */
  int64_t oob;             /* proposals outside the prior box (not evaluated)           */
  int64_t stepout_caps;    /* stepping-out sides that hit max_stepout                   */
  int64_t shrink_caps;     /* slice iterations that hit max_shrink                      */
  int64_t clusterings;     /* cluster-tree builds                                       */
  int64_t nan_logL;        /* likelihood values that were NaN (counted as -inf): every
                              NaN a callback returns, and NaNs of the initial points  */
  int32_t done;            /* stopping rule reached                                     */
  int32_t n_clusters;      /* clusters of the current tree                              */
  int64_t screened;        /* proposals the surrogate screened out (not evaluated)      */
  int64_t net_rows;        /* rows evaluated by the likelihood network, speculative
                              rows of the batched rounds included                       */
} ns_stats_t;

/* Defaults listed above. */
ns_status ns_config_default(ns_config* cfg);

/* Create a sampler: N = n_live initial points drawn uniformly in [lo, hi]
 * (Sec. 1), their likelihoods, and the first cluster tree (Sec. 2.1).
 * lo, hi: host arrays of d doubles.  hip_stream: a hipStream_t, or NULL for
 * the default (null) stream.
 * On success *out owns all device memory of the context (freed by ns_free).
 * Debugging aid: with the environment variable NS_FILL_ALLOC=<byte> set, every
 * device buffer the context allocates (here and in later calls) is filled
 * with that byte before first use; results do not change, since no call reads
 * device memory it has not written. */
ns_status ns_init(ns_ctx** out, const double* lo, const double* hi, int d, int n_live,
                  const ns_config* cfg, const ns_likelihood* lik, void* hip_stream);

/* One batched update of m live points (Sec. 3; Algorithms 1 and 2): select the
 * m worst, run m constrained slice-sampling chains, correct, update the live
 * set, append m dead rows and accumulate the evidence.  Enqueued without
 * synchronising; the host follows the device through a progress word in
 * pinned host memory and waits only while more than eight steps are in
 * flight.  Returns NS_DONE once the stopping rule is known to hold (the device
 * checks it after every step; steps after it are no-ops). */
ns_status ns_step_batch(ns_ctx* c, int m);

/* Repeat ns_step_batch(m) until the stopping rule holds or max_steps steps
 * have been enqueued; *steps (may be NULL) = steps that did work.  Returns
 * NS_DONE or NS_OK. */
ns_status ns_run(ns_ctx* c, int m, int64_t max_steps, int64_t* steps);

/* R independent runs at once: ns_run(ctxs[r], m, max_steps, &steps[r]) for
 * every r, each from a host thread of its own, so that the runs' steps are in
 * flight together and the device holds R * m chains.  Independent runs (the
 * alternative to batching that the paper weighs in Sec. 1, and the way to fill
 * the device when m is small) give the same results as run one by one: each
 * context draws from its own seed and runs on its own stream.  For overlap the
 * contexts need distinct streams (ns_init's hip_stream), and the HIP runtime
 * at least R hardware queues (environment GPU_MAX_HW_QUEUES >= R, at most 32,
 * set before the runtime starts; streams beyond it share queues and
 * serialise).  Contexts with a callback likelihood run their callbacks from
 * these threads.  steps (R entries, may be NULL) as in ns_run.  Returns the
 * first error in context order (its ns_last_error describes it), else NS_DONE
 * if every run reached the stopping rule, else NS_OK. */
ns_status ns_run_many(ns_ctx* const* ctxs, int R, int m, int64_t max_steps, int64_t* steps);

/* Wait for all enqueued work of the context. */
ns_status ns_sync(ns_ctx* c);

/* Evidence, Eq. (1) Z = int L(X) dX, by the single-point integration the
 * paper keeps for batched deaths (Sec. 3): dead row i (i = 1, 2, ...) has
 * log X_i = -i/N and the rectangle weight w_i = (X_{i-1} - X_i) L_i; the final
 * live points are added, each with prior volume X_end/N.  Returns logZ,
 * sigma = sqrt(H/N) and the information H = sum_i p_i log L_i - log Z
 * (p_i = w_i/Z), all in FP64.  Does not change the run; any output pointer may
 * be NULL; synchronises the context's stream. */
ns_status ns_logZ(ns_ctx* c, double* logZ, double* sigma, double* H);

/* Dead rows in death order (Algorithm 1: the rejected entries of each batch,
 * ascending).  Two-phase: with u == logL == logX == logw == NULL only *n is
 * set.  Otherwise arrays hold *n rows: u (n*d), logL, logX = -i/N and the
 * rectangle weight logw = log((X_{i-1} - X_i) L_i) of the single-point
 * integration of Eq. (1) (host arrays, any may be NULL). */
ns_status ns_get_dead(ns_ctx* c, int64_t* n, double* u, double* logL, double* logX, double* logw);

/* Live set: u (N*d), logL (N), label (N: cluster node of each point); host
 * arrays, any may be NULL. */
ns_status ns_get_live(ns_ctx* c, double* u, double* logL, int* label);

/* Replace the live set (host arrays u N*d, logL N, label N; label may be NULL
 * to keep the labels).  Points are rounded to the state precision. */
ns_status ns_set_live(ns_ctx* c, const double* u, const double* logL, const int* label);

/* Cluster tree (Sec. 2.1), heap indexed, n_nodes = 2^(D+1)-1.  Host arrays:
 * count, accepted (1 = cluster of the pruned tree), split_ok (n_nodes ints),
 * logV (n_nodes), centre (n_nodes*d), chol (n_nodes*d*d, lower triangle of the
 * regularised covariance's Cholesky factor).  Any may be NULL. */
ns_status ns_get_tree(ns_ctx* c, int* n_nodes, int* count, int* accepted, int* split_ok,
                      double* logV, double* centre, double* chol);

/* Inputs and outputs of the last enqueued step (for parity checks): *m = its
 * batch size; seeds (m slots),
 * tau (m thresholds), new_u (m*d) and new_logL (m) of the chains before the
 * correction, chain_evals (m), hist_logL (T*m, row t = shrink proposal t of
 * the last slice iteration, slot T-1 = the chain's final point), hist_u
 * (m*T*d), hist_n (m recorded proposals).  Host arrays, any may be NULL. */
ns_status ns_get_last_batch(ns_ctx* c, int* m, int* seeds, double* tau, double* new_u,
                            double* new_logL, int64_t* chain_evals, double* hist_logL,
                            double* hist_u, int* hist_n);

/* Counters; synchronises. */
ns_status ns_stats(ns_ctx* c, ns_stats_t* s);

/* Evaluate the context's likelihood, as the sampler does, at n unit-cube
 * points: d_u device array n*d doubles (rounded to the state precision first),
 * d_out device array n doubles.  Enqueued on the context's stream. */
ns_status ns_loglike_batch(ns_ctx* c, const double* d_u, int64_t n, double* d_out);

/* Algorithm 1 "sorted": ascending order of (logL, slot) of N keys (NaN counts
 * as -inf, -0 as +0).  d_logL: N doubles, d_order: N ints (device).  N <= 8192. */
ns_status ns_select_order(const double* d_logL, int N, int* d_order, void* hip_stream);

/* Algorithm 1 "sorted" at scale: the m entries with the smallest (logL, index)
 * (NaN counts as -inf, -0 as +0), ascending, the same order as the first m of
 * ns_select_order, for 1 <= N <= 2^31 - 1 and 1 <= m <= min(N, 4096).  A
 * radix select over the FP64 order key (and, for ties, the index) makes one
 * streaming pass over d_logL per resolved 12-bit digit until at most 8192
 * entries remain at or below the resolved prefix, then one collect pass and
 * a sort of those candidates.  d_logL: N doubles, 16-byte aligned (device);
 * d_slots: m ints (device, written); d_work: ns_select_worst_work_bytes()
 * bytes of device workspace, 256-byte aligned, caller-owned, overwritten
 * (calls that overlap in time must not share it); d_passes (device, may be
 * NULL): receives the number of passes made over d_logL.  Enqueued on
 * hip_stream; NS_EINVAL on bad sizes or alignment. */
size_t ns_select_worst_work_bytes(void);
/* One node of the cluster tree (Sec. 2.1) for large point sets: mean,
 * unbiased covariance and the k-means split (k = 2; start at the point
 * farthest from the mean and the point farthest from that one, lowest index
 * on ties; a point joins the first centre on a distance tie; Lloyd updates
 * until no assignment changes or after iters updates; an empty side keeps its
 * centre), as the tree kernels compute them per node, for 2 <= N <= 2^31 - 1
 * and 1 <= d <= 32.  Every statistic is one streaming pass over d_u.  d_u:
 * N x d FP32, row major (device); d_mean: d doubles; d_cov: d x d doubles
 * (row stride d); d_centres: 2 x 32 doubles (row 0 the first centre);
 * d_side: N bytes (0 or 1); d_work: ns_cluster_split_work_bytes() bytes of
 * device workspace, 256-byte aligned, caller-owned (calls that overlap in time
 * must not share it); d_passes (may be NULL): passes made over d_u.  Enqueued
 * on hip_stream; NS_EINVAL on bad sizes or alignment. */
size_t ns_cluster_split_work_bytes(void);
ns_status ns_cluster_split(const float* d_u, int64_t N, int d, int iters, double* d_mean, double* d_cov,
                           double* d_centres, uint8_t* d_side, void* d_work, int* d_passes, void* hip_stream);
ns_status ns_select_worst(const double* d_logL, int64_t N, int m, int* d_slots, void* d_work, int* d_passes,
                          void* hip_stream);

/* The same selection as ns_select_worst, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no workspace argument, and no allocation in the
 * call.  The workspace is a static device array of ns_select_worst_work_bytes()
 * bytes (about 8.5 MB) per device, held until the process ends; its address
 * is looked up on the first call on a device.  Limits: 1 <= m <= min(N, 4096),
 * N <= 2^31 - 1 (NS_EINVAL beyond, with the reason in ns_last_error(NULL)).
 * d_logL (16-byte aligned), d_slots and d_passes (may be NULL) as in
 * ns_select_worst, on the current device; hip_stream (NULL: the default
 * stream) must belong to the current device.  All calls on one device share
 * the workspace: calls that overlap in time on one device race, and the
 * caller must order them (one stream, or events). */
ns_status ns_select_worst_noalloc(const double* d_logL, int64_t N, int m, int* d_slots, int* d_passes,
                                  void* hip_stream);

/* Algorithms 1 and 2 on explicit arrays (device): d_wlogL (m, ascending),
 * d_nlogL (m), d_P (m thresholds), d_hist (T*m, row t, column = chain),
 * d_hist_n (m).  Outputs (device, m each): accepted and rejected entries as
 * codes (< m: worst point, >= m: chain code-m), history slot (-1: the chain's
 * final point) and logL, each ascending.  m <= 1024. */
ns_status ns_correct_batch(int m, ns_corr corr, int K, int T, const double* d_wlogL,
                           const double* d_nlogL, const double* d_P, const double* d_hist,
                           const int* d_hist_n, int* d_acc_code, int* d_acc_hslot,
                           double* d_acc_logL, int* d_rej_code, int* d_rej_hslot,
                           double* d_rej_logL, void* hip_stream);

/* The generator the sampler draws from: Philox4x32-10 (Salmon et al., SC'11)
 * evaluated on the device for n counters {c0 + k, c1, c2, c3}, k < n, key =
 * seed; d_out receives 4n words.  Exposed so the stream can be checked. */
ns_status ns_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                    int64_t n, uint32_t* d_out, void* hip_stream);

/* Per-kernel-class device time, measured with HIP events recorded on the
 * context's stream around each launch sequence: classes NS_TIME_SELECT
 * (sort + seeds), NS_TIME_SLICE (the chains), NS_TIME_CORRECT (Algorithms
 * 1/2, update, evidence), NS_TIME_CLUSTER (tree build), NS_TIME_DRAWS (the
 * draw pre-pass of the fused slice kernel).  ns_set_timing(c, mask)
 * clears the counters and times the classes whose bit (1 << class) is set in
 * mask (NS_TIMING_ALL for every class, 0 for none); each timed launch
 * sequence adds two event records to the stream.  ns_get_timing synchronises
 * and returns total milliseconds and launch counts per class (arrays of
 * NS_TIMING_CLASSES, may be NULL; untimed classes read zero).  NS_TIME_LIK:
 * the batched likelihood kernels of the rounds (network layers and chi^2). */
#define NS_TIMING_CLASSES 6
#define NS_TIME_SELECT 0
#define NS_TIME_SLICE 1   /* fused slice kernel, or the chain kernels of batched rounds */
#define NS_TIME_CORRECT 2
#define NS_TIME_CLUSTER 3
#define NS_TIME_LIK 4     /* batched likelihood of the rounds (network layers, chi^2)  */
#define NS_TIME_DRAWS 5   /* directions and uniforms of the fused slice kernel        */
#define NS_TIMING_ALL 0x3F
ns_status ns_set_timing(ns_ctx* c, int mask);
ns_status ns_get_timing(ns_ctx* c, double* ms, int64_t* launches);

/* ---- dense networks (emulator likelihood, learned surrogate) --------------
 * A fully connected network y = f(x): layer l maps widths[l] -> widths[l+1]
 * as z = h W_l + b_l, hidden layers apply act (NS_ACT_TANH or NS_ACT_SILU),
 * the output layer is linear.  Weights and biases are caller-owned device
 * arrays (FP32, W_l row major widths[l] x widths[l+1]).  prec: NS_FP32 (FMA
 * on the vector ALU), NS_BF16 (MFMA with FP32 accumulation; operands rounded
 * to bfloat16) or NS_BF16X3 (weights rounded to bfloat16, activations split
 * in three bfloat16 terms).  The surrogate of the sampler's own (theta, logL)
 * pairs is trained with these two calls (behind torch.autograd.Function). */
#define NS_ACT_TANH 1
#define NS_ACT_SILU 2
typedef struct {
  int n_layers;            /* 1..8 */
  int widths[9];
  int act;
  const float* W[8];
  const float* b[8];
} ns_mlp_desc;

/* Forward pass of B rows: d_X (B x widths[0]), d_Y (B x widths[L]).  d_Z
 * (may be NULL) receives every layer's pre-activation, layer l at offset
 * B * (widths[1] + ... + widths[l]); d_H (may be NULL) every hidden layer's
 * output at the same offsets (the last block unused). */
ns_status ns_mlp_forward(const ns_mlp_desc* net, ns_prec prec, const float* d_X, int64_t B,
                         float* d_Y, float* d_Z, float* d_H, void* hip_stream);

/* Backward pass for the loss gradient d_dY (B x widths[L]), given the d_Z and
 * d_H of the forward pass: d_dW[l] (widths[l] x widths[l+1]) and d_db[l]
 * receive dLoss/dW_l and dLoss/db_l (overwritten), d_dX (may be NULL)
 * dLoss/dX.  d_work: 2 * B * max(widths) floats of scratch. */
ns_status ns_mlp_backward(const ns_mlp_desc* net, ns_prec prec, const float* d_X, int64_t B,
                          const float* d_Z, const float* d_H, const float* d_dY,
                          float* const* d_dW, float* const* d_db, float* d_dX, float* d_work,
                          void* hip_stream);

/* ---- learned pre-screen (network likelihoods) -------------------------------
 * A small surrogate network widths {d, hidden, hidden, 1} with SiLU hidden
 * layers, trained on the device on the (theta, logL) pairs the sampler itself
 * evaluates (replay ring), with the kernels of ns_mlp_forward/backward, an MSE
 * loss and Adam.  Targets t = max(logL, L_W[0] - floor_below) are mapped
 * linearly from [L_W[0] - floor_below, best live logL] to [-1, 1]; inputs are
 * standardised with the live set's mean and standard deviation.  Once
 * min_pairs pairs are stored training starts, and while the last minibatch's
 * RMS error is below margin/2 nats each round's proposals are scored:
 * a proposal whose estimate lies below its threshold minus `margin` is taken
 * as failing without evaluating the true likelihood, except every
 * audit_period-th such proposal, which is evaluated; if a step's audited
 * false-screen rate exceeds max_fn_rate the screen pauses for five steps
 * (plain sampler as fallback).  Accepted points always carry their true
 * likelihood.  Only for NS_LIK_MLP contexts. */
typedef struct {
  int hidden;            /* 256 */
  int replay_cap;        /* 65536 pairs */
  int batch;             /* 2048 */
  int train_every;       /* steps between training calls; 1 */
  int train_iters;       /* Adam steps per call; 25 */
  float lr;              /* 1e-3 */
  double margin;         /* nats; 5 */
  double floor_below;    /* nats; 40 */
  int audit_period;      /* 16 */
  double max_fn_rate;    /* 0.02 */
  int min_pairs;         /* 16384 */
  ns_prec prec;          /* NS_FP32 or NS_BF16 layers; NS_BF16 */
  uint64_t seed;
} ns_surrogate_config;

typedef struct {
  int64_t pairs;          /* pairs appended to the replay ring                     */
  int64_t net_rows;       /* true-likelihood network rows                          */
  int64_t screened;       /* proposals the surrogate placed below threshold-margin */
  int64_t audited;
  int64_t false_screens;
  int64_t train_calls;
  int32_t screening;      /* screen active now                                      */
  int32_t disabled;       /* paused by the audit                                    */
  double last_loss;       /* MSE of the last minibatch (normalised units)           */
} ns_surrogate_stats_t;

ns_status ns_surrogate_default(ns_surrogate_config* sc);
ns_status ns_surrogate_enable(ns_ctx* c, const ns_surrogate_config* sc);
ns_status ns_surrogate_stats(ns_ctx* c, ns_surrogate_stats_t* s);
/* logL estimate of n points d_theta (n*d FP32 parameter values, device) into
 * d_out (n FP32). */
ns_status ns_surrogate_predict(ns_ctx* c, const float* d_theta, int64_t n, float* d_out);

/* Description of the last error of c (or of the last context-free call when
 * c is NULL); valid until the next call on c. */
const char* ns_last_error(const ns_ctx* c);

/* Release the context and all its device memory.  NULL-safe. */
void ns_free(ns_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
