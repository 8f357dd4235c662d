/*
 * ns_oracle.h -- plain, slow, FP64 CPU oracle of the batched nested sampler of
 * "Fast and efficient nested sampling with BEST" (arXiv 2608.28514).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; the two are written independently from
 * the paper and from the algorithm statement below.
 *
 * Everything is FP64 and written as plain loops in the order the paper states
 * the steps: Eq. (1) and the single-point evidence integration (Sec. 1, 3),
 * k-means cluster tree with volume pruning and eigenvalue-clipped covariances
 * (Sec. 2.1), slice sampling along covariance-transformed directions (Sec. 2.2),
 * batch sorting (Algorithm 1) and history correction (Algorithm 2, Sec. 3.1).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
 * the run seed, counter = (draw, item, step, stream<<24 | sub).  See the stream
 * constants below; the GPU library implements the same published generator.
 *
 * Parity status per function is listed in the header comment of each source.
 */
#ifndef NS_ORACLE_H
#define NS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXD 32
#define ORC_MAX_DEPTH 6

/* Philox counter word 3 = stream << 24 | sub-index. */
enum {
  ORC_STREAM_INIT = 1,   /* c0 = pair index, c1 = live point, c2 = 0          */
  ORC_STREAM_SEED = 2,   /* c0 = 0,          c1 = chain,      c2 = step       */
  ORC_STREAM_SLICE = 3   /* c0 = draw slot,  c1 = chain,      c2 = step, sub = slice iteration */
};
/* draw slots inside one slice iteration */
#define ORC_SLOT_DIR0 0u      /* direction pairs 0..15                       */
#define ORC_SLOT_STEPOUT 16u  /* initial bracket offset                      */
#define ORC_SLOT_SHRINK0 32u  /* shrink attempt s uses slot 32+s             */

enum { ORC_LIK_MIXTURE = 0, ORC_LIK_ROSENBROCK = 1, ORC_LIK_SHELL = 2, ORC_LIK_MLP = 3 };
enum { ORC_CORR_NONE = 0, ORC_CORR_BEST_OF_WORST = 1, ORC_CORR_SORT = 2, ORC_CORR_HISTORY = 3 };

typedef struct {
  int kind;
  int d;
  /* mixture of axis-aligned Gaussians: logL = logsumexp_k(logw_k - q_k/2),
     q_k = sum_i (theta_i - mu_ki)^2 * ivar_ki                                 */
  int n_comp;
  const double* logw;   /* K       */
  const double* mu;     /* K x d   */
  const double* ivar;   /* K x d   */
  /* Rosenbrock chain: -sum_i [ b (x_{i+1} - x_i^2)^2 + (a - x_i)^2 ]          */
  double ros_a, ros_b;
  /* Gaussian shell: -((|x| - r0) / w)^2 / 2                                    */
  double shell_r0, shell_w;
  /* MLP emulator: tanh hidden layers, linear output, diagonal chi^2           */
  int n_layers;            /* number of weight matrices                        */
  const int* widths;       /* n_layers + 1 entries, widths[0] == d             */
  const double* weights;   /* concatenated row-major W_l (widths[l] x widths[l+1]) */
  const double* biases;    /* concatenated b_l (widths[l+1])                   */
  const double* data;      /* widths[n_layers]                                 */
  const double* sigma;     /* widths[n_layers]                                 */
} orc_lik;

typedef struct {
  int slice_steps_per_dim;  /* n: n*d slice iterations per chain (Sec. 2.2)   */
  double step_width;        /* w: bracket width in direction units            */
  int max_stepout;          /* E_max per side                                 */
  int max_shrink;           /* S_max                                          */
  int tree_depth;           /* D: at most 2^D clusters (Sec. 2.1)             */
  double split_vol_frac;    /* p: children must be p*100 % smaller            */
  int min_cluster_pts;      /* n_min: both children need more points; 0 => 2(d+1) */
  int recluster_every;      /* R deaths between clusterings                   */
  int kmeans_iters;         /* Lloyd iteration cap                            */
  int correction;           /* ORC_CORR_*                                     */
  int history_iters;        /* K of Algorithm 2                               */
  int hist_cap;             /* T: stored shrink proposals of the last iteration */
  double stop_frac;         /* remaining-evidence fraction that stops the run */
  double eig_floor;         /* relative eigenvalue floor of the clip          */
  uint64_t seed;
} orc_config;

typedef struct orc_ctx orc_ctx;

/* ---- random numbers -------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* the two uniforms in (0,1) of one Philox call */
void orc_uniform2(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double out[2]);

/* ---- likelihood ------------------------------------------------------------ */
/* u: n x d unit-cube points; theta = lo + (hi-lo) u.  Out-of-box => -inf, NaN => -inf. */
void orc_loglike(const orc_lik* L, const double* lo, const double* hi,
                 const double* u, long n, double* out);

/* ---- selection (Algorithm 1, "sorted") ------------------------------------- */
/* ascending order of (logL, slot); NaN counts as -inf, -0 as +0 */
void orc_select(const double* logL, int N, int* order);

/* ---- linear algebra and clustering (Sec. 2.1) ------------------------------ */
int orc_jacobi_eig(int d, const double* A, double* evals, double* evecs);
int orc_cholesky(int d, const double* A, double* L);
/* k-means split (k = 2) of n points u (n x d), as one tree node: side[k] and
 * the final centres ca, cb (d each). */
void orc_two_means(const double* u, int n, int d, int iters, double* ca, double* cb, int* side);
/* eigen-clip + Cholesky; returns log volume sum log L_ii, writes L */
double orc_regularise(int d, const double* cov, double eps, double* Lout, int* clipped);

typedef struct {
  int depth, d, n_nodes;
  int count[127];
  int split_ok[127];       /* node kept its two children after pruning     */
  int accepted[127];       /* node is a cluster of the pruned tree          */
  double logV[127];
  double logV_eff[127];
  double centre[127 * ORC_MAXD];
  double chol[127 * ORC_MAXD * ORC_MAXD];
} orc_tree;

int orc_cluster(const double* u, int N, int d, int depth, double p, int nmin,
                int kmeans_iters, double eps, orc_tree* tree, int* labels);
int orc_nearest_centre(const orc_tree* t, const double* x);

/* ---- batch correction (Algorithms 1 and 2) --------------------------------- */
/* Inputs: W logL (m, ascending), new-point logL (m), their thresholds P (m),
   history logL (T x m, column j = chain j, entries past hist_n[j] unused, slot
   T-1 = accepted), hist_n (m).  Outputs: acc/rej entries as codes: code < m is
   W entry code, code >= m is chain (code-m) with history slot hslot (-1: its
   final point).  acc_logL/rej_logL the logL of each entry (ascending). */
int orc_correct(int m, int corr, int K, int T,
                const double* wlogL, const double* nlogL, const double* P,
                const double* hist, const int* hist_n,
                int* acc_code, int* acc_hslot, double* acc_logL,
                int* rej_code, int* rej_hslot, double* rej_logL);

/* ---- sampler context ------------------------------------------------------- */
void orc_config_default(orc_config* c);
orc_ctx* orc_create(const double* lo, const double* hi, int d, int N,
                    const orc_config* cfg, const orc_lik* lik);
void orc_free(orc_ctx* c);
int orc_step(orc_ctx* c, int m);                 /* 1 once the stop rule holds */
long orc_run(orc_ctx* c, int m, long max_steps);  /* steps that did work        */
void orc_logZ(orc_ctx* c, double* logZ, double* sigma, double* H);
long orc_n_dead(const orc_ctx* c);
void orc_get_dead(const orc_ctx* c, double* u, double* logL, double* logX, double* logw);
void orc_get_live(const orc_ctx* c, double* u, double* logL, int* label);
void orc_set_live(orc_ctx* c, const double* u, const double* logL, const int* label);
void orc_get_tree(const orc_ctx* c, orc_tree* t);
void orc_set_tree(orc_ctx* c, const orc_tree* t);
void orc_get_counters(const orc_ctx* c, long* out8);  /* evals, oob, stepout caps, shrink caps, steps, dead, nan, clusterings */
void orc_get_state(const orc_ctx* c, double* logZ_run, double* A_run, long* step, int* done);
/* last step: seeds, thresholds, new points / logL / chain evals, history */
void orc_get_last_batch(const orc_ctx* c, int* seeds, double* tau, double* new_u, double* new_logL,
                        long* chain_evals, double* hist_logL, double* hist_u, int* hist_n);
/* last step, per chain: the start point x0 and direction v of the last slice
   iteration and its stepped-out bracket [a, b] (ka, kb steps per side), before
   shrinking (test hooks) */
void orc_get_last_brackets(const orc_ctx* c, double* x0, double* v, double* a, double* b, int* ka, int* kb);
/* direction v = L zhat of slice iteration `it` of chain j (Sec. 2.2); L lower
   triangular, row stride ORC_MAXD */
void orc_slice_direction(uint64_t seed, int j, uint32_t step, int it, const double* L, int d, double* v);
void orc_set_threads(int n);
int orc_get_threads(void);

/* ---- MLP (surrogate training) -------------------------------------------- */
/* act: 0 tanh, 1 SiLU; hidden layers use act, output layer is linear. */
void orc_mlp_forward(int n_layers, const int* widths, const double* W, const double* b,
                     int act, const double* X, long B, double* Y, double* acts);
void orc_mlp_backward(int n_layers, const int* widths, const double* W, const double* b,
                      int act, const double* X, long B, const double* acts, const double* dY,
                      double* dW, double* db, double* dX);

#ifdef __cplusplus
}
#endif
#endif
