/*
 * sampler.c -- the batched nested sampler, step by step, in FP64.
 * TEST INFRASTRUCTURE (oracle): only tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.
 *
 * One step of orc_step(m) is, in the paper's order:
 *   1. (re)cluster the live points when R deaths have passed   (Sec. 2.1)
 *   2. sort the live points by likelihood, W = the m worst      (Algorithm 1)
 *   3. choose a seed for each of the m chains                   (Algorithm 1, RNG.choose)
 *   4. slice sampling, n*d iterations per chain, hard
 *      constraint logL > L_W[j]; the bracket is stepped out
 *      against the batch-worst L_W[0]; the shrink proposals of
 *      the last iteration are kept as history                  (Sec. 2.2, Sec. 3.1)
 *   5. naive / best-of-worst / batch sorting / history correction
 *                                                               (Sec. 3, Algorithms 1 and 2)
 *   6. accepted points replace the worst, rejected points die   (Algorithm 1)
 *   7. single-point evidence integration of the dead points and
 *      the stopping rule                                        (Eq. (1), Sec. 3)
 *
 * Readings of what the paper leaves open (all shared with the GPU library
 * through the written algorithm statement only, never through code):
 *  - every dead row is one sequential death, log X_i = -i/N, and carries the
 *    rectangle weight (X_{i-1} - X_i) L_i; the final live points share X_end;
 *  - stop once X_i * max(L_live) < stop_frac * Z_i, checked after each step;
 *  - seeds: chain j starts from a uniformly chosen point ranked above W[j];
 *  - directions: v = L_c zhat, zhat uniform on the sphere, L_c the Cholesky
 *    factor of the seed's cluster, kept for the whole chain; bracket width w
 *    in units of v, linear stepping out to E_max per side, at most S_max
 *    shrinks; strict ">" for every constraint;
 *  - the stepped-out offsets are a0 - k w and b0 + k w, computed directly;
 *  - history: the first T-1 shrink proposals of the last iteration, plus the
 *    accepted point in slot T-1;
 *  - ties in every sort are broken by the original position; NaN logL counts
 *    as -inf; -0 equals +0;
 *  - accepted new points fill the slots of rejected worst points in the order
 *    of W; revived worst points keep their slots.
 *
 * Pins: tests/test_oracle_sampler.py and tests/test_oracle_correct.py (worked
 * examples of Algorithms 1 and 2, constant likelihood gives log Z = c exactly,
 * log X_i = -i/N, monotone dead likelihoods under sorting corrections, m = 1
 * identical for every correction, closed-form log Z of Gaussian and mixture
 * runs, uniformity of slice output inside a spherical constraint, exact replay
 * of the history relaxation) and tests/test_oracle_pins.py (brackets stepped
 * out against L_W[0] while shrinking uses L_W[j], seed ranks uniform above
 * W[j], v = L_c zhat with zhat uniform on the sphere, 2-d Rosenbrock evidence
 * against quadrature to 3 standard errors, sequential and batched).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include "ns_oracle.h"

/* bracket of the last slice iteration of a chain, as stepped out (test hooks) */
typedef struct {
  double x0[ORC_MAXD], v[ORC_MAXD];
  double a, b;
  int ka, kb;
} last_bracket;

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

void orc_config_default(orc_config* c) {
  c->slice_steps_per_dim = 5;
  c->step_width = 1.0;
  c->max_stepout = 64;
  c->max_shrink = 64;
  c->tree_depth = 0;
  c->split_vol_frac = 0.3;
  c->min_cluster_pts = 0;
  c->recluster_every = 100;
  c->kmeans_iters = 20;
  c->correction = ORC_CORR_HISTORY;
  c->history_iters = 1;
  c->hist_cap = 32;
  c->stop_frac = 1e-3;
  c->eig_floor = 1e-8;
  c->seed = 0;
}

struct orc_ctx {
  int d, N, nmin;
  double lo[ORC_MAXD], hi[ORC_MAXD];
  orc_config cfg;
  orc_lik lik;
  /* owned copies of likelihood parameters */
  double *p_logw, *p_mu, *p_ivar, *p_W, *p_b, *p_data, *p_sigma;
  int* p_widths;
  /* live set */
  double* u;
  double* logL;
  int* label;
  orc_tree tree;
  /* evidence */
  long n_dead;
  double logZ, A;
  long step;
  int done;
  long since_cluster;
  /* dead store */
  double *dead_u, *dead_logL;
  long dead_cap;
  /* counters */
  long evals, oob, so_caps, sh_caps, clusterings;
  /* last batch */
  int last_m;
  int* seeds;
  double* tau;
  double* new_u;
  double* new_logL;
  long* chain_evals;
  double* hist_logL;
  double* hist_u;
  int* hist_n;
  last_bracket* brk;
  int cap_m;
};

static double* dup_d(const double* p, long n) {
  if (!p || n <= 0) return NULL;
  double* q = (double*)malloc(sizeof(double) * n);
  memcpy(q, p, sizeof(double) * n);
  return q;
}

static void loglike_pts(orc_ctx* c, const double* u, long n, double* out) {
  orc_loglike(&c->lik, c->lo, c->hi, u, n, out);
}

static double loglike1(orc_ctx* c, const double* y) {
  double v;
  orc_loglike(&c->lik, c->lo, c->hi, y, 1, &v);
  return v;
}

static void recluster(orc_ctx* c) {
  orc_cluster(c->u, c->N, c->d, c->cfg.tree_depth, c->cfg.split_vol_frac, c->nmin,
              c->cfg.kmeans_iters, c->cfg.eig_floor, &c->tree, c->label);
  c->since_cluster = 0;
  c->clusterings++;
}

orc_ctx* orc_create(const double* lo, const double* hi, int d, int N,
                    const orc_config* cfg, const orc_lik* lik) {
  if (d < 1 || d > ORC_MAXD || N < 2) return NULL;
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->d = d;
  c->N = N;
  c->cfg = *cfg;
  c->nmin = cfg->min_cluster_pts > 0 ? cfg->min_cluster_pts : 2 * (d + 1);
  for (int i = 0; i < d; ++i) { c->lo[i] = lo[i]; c->hi[i] = hi[i]; }
  c->lik = *lik;
  c->lik.d = d;
  if (lik->kind == ORC_LIK_MIXTURE) {
    c->p_logw = dup_d(lik->logw, lik->n_comp);
    c->p_mu = dup_d(lik->mu, (long)lik->n_comp * d);
    c->p_ivar = dup_d(lik->ivar, (long)lik->n_comp * d);
    c->lik.logw = c->p_logw; c->lik.mu = c->p_mu; c->lik.ivar = c->p_ivar;
  } else if (lik->kind == ORC_LIK_MLP) {
    int L = lik->n_layers;
    c->p_widths = (int*)malloc(sizeof(int) * (L + 1));
    memcpy(c->p_widths, lik->widths, sizeof(int) * (L + 1));
    long nw = 0, nb = 0;
    for (int l = 0; l < L; ++l) { nw += (long)lik->widths[l] * lik->widths[l + 1]; nb += lik->widths[l + 1]; }
    c->p_W = dup_d(lik->weights, nw);
    c->p_b = dup_d(lik->biases, nb);
    c->p_data = dup_d(lik->data, lik->widths[L]);
    c->p_sigma = dup_d(lik->sigma, lik->widths[L]);
    c->lik.widths = c->p_widths; c->lik.weights = c->p_W; c->lik.biases = c->p_b;
    c->lik.data = c->p_data; c->lik.sigma = c->p_sigma;
  }
  c->u = (double*)malloc(sizeof(double) * N * d);
  c->logL = (double*)malloc(sizeof(double) * N);
  c->label = (int*)calloc(N, sizeof(int));
  /* initial live points: uniform draws in the prior box */
  for (int k = 0; k < N; ++k)
    for (int p = 0; 2 * p < d; ++p) {
      double w[2];
      orc_uniform2(cfg->seed, (uint32_t)p, (uint32_t)k, 0u, (uint32_t)ORC_STREAM_INIT << 24, w);
      c->u[(long)k * d + 2 * p] = w[0];
      if (2 * p + 1 < d) c->u[(long)k * d + 2 * p + 1] = w[1];
    }
  loglike_pts(c, c->u, N, c->logL);
  c->evals = N;
  c->logZ = -INFINITY;
  c->A = 0.0;
  recluster(c);
  c->clusterings = 1;
  return c;
}

void orc_free(orc_ctx* c) {
  if (!c) return;
  free(c->p_logw); free(c->p_mu); free(c->p_ivar); free(c->p_W); free(c->p_b);
  free(c->p_data); free(c->p_sigma); free(c->p_widths);
  free(c->u); free(c->logL); free(c->label);
  free(c->dead_u); free(c->dead_logL);
  free(c->seeds); free(c->tau); free(c->new_u); free(c->new_logL); free(c->chain_evals);
  free(c->hist_logL); free(c->hist_u); free(c->hist_n); free(c->brk);
  free(c);
}

/* ---- selection ------------------------------------------------------------- */
static const double* g_sort_keys;
static double canon(double x) { return isnan(x) ? -INFINITY : (x == 0.0 ? 0.0 : x); }
static int cmp_slot(const void* a, const void* b) {
  int i = *(const int*)a, j = *(const int*)b;
  double x = canon(g_sort_keys[i]), y = canon(g_sort_keys[j]);
  if (x < y) return -1;
  if (x > y) return 1;
  return (i > j) - (i < j);
}
void orc_select(const double* logL, int N, int* order) {
  for (int k = 0; k < N; ++k) order[k] = k;
  g_sort_keys = logL;
  qsort(order, N, sizeof(int), cmp_slot);
}

/* ---- slice sampling of one chain (Sec. 2.2) ------------------------------- */
typedef struct {
  long evals, oob, so_caps, sh_caps;
} chain_stats;

static int inbox(int d, const double* y) {
  for (int i = 0; i < d; ++i) if (!(y[i] >= 0.0 && y[i] <= 1.0)) return 0;
  return 1;
}

/* Direction of slice iteration `it` of chain j in step `step` (Sec. 2.2): an
 * isotropic direction zhat (Box-Muller normals, normalised), transformed with
 * the lower-triangular Cholesky factor L (row stride ORC_MAXD) of the chain's
 * cluster covariance: v = L zhat. */
void orc_slice_direction(uint64_t seed, int j, uint32_t step, int it, const double* L, int d, double* v) {
  const uint32_t c3 = ((uint32_t)ORC_STREAM_SLICE << 24) | (uint32_t)it;
  double z[ORC_MAXD];
  for (int p = 0; 2 * p < d; ++p) {
    double uu[2];
    orc_uniform2(seed, ORC_SLOT_DIR0 + (uint32_t)p, (uint32_t)j, step, c3, uu);
    double r = sqrt(-2.0 * log(uu[0]));
    double ang = 6.283185307179586 * uu[1];
    z[2 * p] = r * cos(ang);
    if (2 * p + 1 < d) z[2 * p + 1] = r * sin(ang);
  }
  double nrm = 0.0;
  for (int i = 0; i < d; ++i) nrm += z[i] * z[i];
  nrm = sqrt(nrm);
  for (int i = 0; i < d; ++i) z[i] = z[i] / nrm;
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += L[i * ORC_MAXD + k] * z[k];
    v[i] = s;
  }
}

static void slice_chain(orc_ctx* c, int j, int seed_slot, double tau_j, double tau_e,
                        double* xout, double* lout, double* hl, double* hu, int* hn,
                        chain_stats* st, last_bracket* lb) {
  const int d = c->d, n_iter = c->cfg.slice_steps_per_dim * d, T = c->cfg.hist_cap;
  const double w = c->cfg.step_width;
  const uint64_t seed = c->cfg.seed;
  const uint32_t step = (uint32_t)c->step;
  double x[ORC_MAXD], y[ORC_MAXD], v[ORC_MAXD];
  memcpy(x, c->u + (long)seed_slot * d, sizeof(double) * d);
  double lx = c->logL[seed_slot];
  const double* L = c->tree.chol + (long)c->label[seed_slot] * ORC_MAXD * ORC_MAXD;
  *hn = 0;
  for (int it = 0; it < n_iter; ++it) {
    const uint32_t c3 = ((uint32_t)ORC_STREAM_SLICE << 24) | (uint32_t)it;
    const int last = (it == n_iter - 1);
    orc_slice_direction(seed, j, step, it, L, d, v);
    /* stepping out against the batch-worst threshold */
    double uu[2];
    orc_uniform2(seed, ORC_SLOT_STEPOUT, (uint32_t)j, step, c3, uu);
    const double a0 = -w * uu[0];
    const double b0 = a0 + w;
    int ka = 0;
    for (;;) {
      if (ka == c->cfg.max_stepout) { st->so_caps++; break; }
      double a = a0 - (double)ka * w;
      for (int i = 0; i < d; ++i) y[i] = x[i] + a * v[i];
      if (!inbox(d, y)) { st->oob++; break; }
      double l = loglike1(c, y);
      st->evals++;
      if (!(l > tau_e)) break;
      ++ka;
    }
    int kb = 0;
    for (;;) {
      if (kb == c->cfg.max_stepout) { st->so_caps++; break; }
      double b = b0 + (double)kb * w;
      for (int i = 0; i < d; ++i) y[i] = x[i] + b * v[i];
      if (!inbox(d, y)) { st->oob++; break; }
      double l = loglike1(c, y);
      st->evals++;
      if (!(l > tau_e)) break;
      ++kb;
    }
    double a = a0 - (double)ka * w;
    double b = b0 + (double)kb * w;
    if (last) {
      memcpy(lb->x0, x, sizeof(double) * d);
      memcpy(lb->v, v, sizeof(double) * d);
      lb->a = a; lb->b = b; lb->ka = ka; lb->kb = kb;
    }
    /* shrinking against the chain's own threshold */
    int acc = 0;
    for (int s = 0; s < c->cfg.max_shrink; ++s) {
      orc_uniform2(seed, ORC_SLOT_SHRINK0 + (uint32_t)s, (uint32_t)j, step, c3, uu);
      double t = a + uu[0] * (b - a);
      for (int i = 0; i < d; ++i) y[i] = x[i] + t * v[i];
      double l;
      if (inbox(d, y)) { l = loglike1(c, y); st->evals++; }
      else { l = -INFINITY; st->oob++; }
      if (last && s < T - 1) {
        hl[s] = l;
        memcpy(hu + (long)s * d, y, sizeof(double) * d);
        *hn = s + 1;
      }
      if (l > tau_j) {
        memcpy(x, y, sizeof(double) * d);
        lx = l;
        acc = 1;
        break;
      }
      if (t < 0.0) a = t; else b = t;
    }
    if (!acc) st->sh_caps++;
  }
  hl[T - 1] = lx;
  memcpy(hu + (long)(T - 1) * d, x, sizeof(double) * d);
  memcpy(xout, x, sizeof(double) * d);
  *lout = lx;
}

/* ---- batch corrections (Algorithms 1 and 2) ------------------------------- */
typedef struct {
  double logL;
  int idx;     /* position in the concatenated set: the sort's tie-break */
  double P;    /* parent threshold                                        */
  int H;       /* chain index, -1 for a worst point                       */
  int code;    /* < m: worst point code; >= m: chain code-m               */
  int hslot;   /* -1: the chain's final point; else history slot          */
} centry;

static int cmp_entry(const void* a, const void* b) {
  const centry* x = (const centry*)a;
  const centry* y = (const centry*)b;
  if (x->logL < y->logL) return -1;
  if (x->logL > y->logL) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

int orc_correct(int m, int corr, int K, int T,
                const double* wlogL, const double* nlogL, const double* P,
                const double* hist, const int* hist_n,
                int* acc_code, int* acc_hslot, double* acc_logL,
                int* rej_code, int* rej_hslot, double* rej_logL) {
  centry* C = (centry*)malloc(sizeof(centry) * 2 * m);
  for (int k = 0; k < m; ++k) {
    C[k].logL = canon(wlogL[k]); C[k].idx = k; C[k].P = -1.0; C[k].H = -1; C[k].code = k; C[k].hslot = -1;
  }
  for (int j = 0; j < m; ++j) {
    centry* e = &C[m + j];
    e->logL = canon(nlogL[j]); e->idx = m + j; e->P = P[j]; e->H = j; e->code = m + j; e->hslot = -1;
  }
  if (corr == ORC_CORR_SORT || corr == ORC_CORR_HISTORY) {
    qsort(C, 2 * m, sizeof(centry), cmp_entry);
    if (corr == ORC_CORR_HISTORY) {
      double* Ibar = (double*)malloc(sizeof(double) * m);
      int* JF = (int*)malloc(sizeof(int) * m);
      for (int k = 0; k < K; ++k) {
        centry* rej = C;
        centry* acc = C + m;
        int nf = 0;
        for (int a = 0; a < m; ++a)
          if (acc[a].H >= 0 && acc[a].P >= acc[0].logL) JF[nf++] = a;
        if (nf == 0) break;
        int ni = 0;
        for (int r = 0; r < m; ++r)
          if (rej[r].H >= 0) Ibar[ni++] = rej[r].logL;  /* already ascending */
        int npair = nf < ni ? nf : ni;
        for (int i = 0; i < npair; ++i) {
          centry* e = &acc[JF[i]];
          int col = e->H;
          double thr = Ibar[i];
          int hit = T - 1;
          for (int t = 0; t < hist_n[col]; ++t)
            if (hist[(long)t * m + col] > thr) { hit = t; break; }
          e->logL = canon(hist[(long)hit * m + col]);
          e->hslot = hit;
          e->P = thr;
        }
        /* re-concatenate [rejected, accepted] and sort again */
        for (int q = 0; q < 2 * m; ++q) C[q].idx = q;
        qsort(C, 2 * m, sizeof(centry), cmp_entry);
      }
      free(Ibar);
      free(JF);
    }
  }
  for (int q = 0; q < m; ++q) {
    rej_code[q] = C[q].code; rej_hslot[q] = C[q].hslot; rej_logL[q] = C[q].logL;
    acc_code[q] = C[m + q].code; acc_hslot[q] = C[m + q].hslot; acc_logL[q] = C[m + q].logL;
  }
  free(C);
  return 0;
}

/* ---- evidence ------------------------------------------------------------- */
static double logaddexp(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  double mx = a > b ? a : b;
  return mx + log1p(exp(-fabs(a - b)));
}

/* add one sample with log weight lw and log-likelihood l to (logZ, A), A being
   the Z-weighted mean of logL */
static void evid_add(double* logZ, double* A, double lw, double l) {
  if (lw == -INFINITY) return;
  double nz = logaddexp(*logZ, lw);
  double keep = (*logZ == -INFINITY) ? 0.0 : *A * exp(*logZ - nz);
  *A = keep + l * exp(lw - nz);
  *logZ = nz;
}

static void dead_push(orc_ctx* c, const double* x, double l) {
  if (c->n_dead >= c->dead_cap) {
    long nc = c->dead_cap ? 2 * c->dead_cap : 4096;
    c->dead_u = (double*)realloc(c->dead_u, sizeof(double) * nc * c->d);
    c->dead_logL = (double*)realloc(c->dead_logL, sizeof(double) * nc);
    c->dead_cap = nc;
  }
  memcpy(c->dead_u + c->n_dead * c->d, x, sizeof(double) * c->d);
  c->dead_logL[c->n_dead] = l;
  const double N = (double)c->N;
  const double lw0 = log(-expm1(-1.0 / N));
  double i = (double)(c->n_dead + 1);
  double lw = (l - (i - 1.0) / N) + lw0;
  evid_add(&c->logZ, &c->A, lw, l);
  c->n_dead++;
}

static void ensure_batch(orc_ctx* c, int m) {
  if (m <= c->cap_m) return;
  const int d = c->d, T = c->cfg.hist_cap;
  free(c->seeds); free(c->tau); free(c->new_u); free(c->new_logL); free(c->chain_evals);
  free(c->hist_logL); free(c->hist_u); free(c->hist_n); free(c->brk);
  c->seeds = (int*)malloc(sizeof(int) * m);
  c->tau = (double*)malloc(sizeof(double) * m);
  c->new_u = (double*)malloc(sizeof(double) * m * d);
  c->new_logL = (double*)malloc(sizeof(double) * m);
  c->chain_evals = (long*)malloc(sizeof(long) * m);
  c->hist_logL = (double*)malloc(sizeof(double) * (long)T * m);
  c->hist_u = (double*)malloc(sizeof(double) * (long)T * m * d);
  c->hist_n = (int*)malloc(sizeof(int) * m);
  c->brk = (last_bracket*)calloc(m, sizeof(last_bracket));
  c->cap_m = m;
}

int orc_step(orc_ctx* c, int m) {
  if (c->done) return 1;
  if (m < 1 || m > c->N - 1) return -1;
  const int d = c->d, N = c->N, T = c->cfg.hist_cap;
  ensure_batch(c, m);
  c->last_m = m;
  if (c->since_cluster >= c->cfg.recluster_every) recluster(c);

  /* sort, worst m, thresholds */
  int* order = (int*)malloc(sizeof(int) * N);
  orc_select(c->logL, N, order);
  double* LW = (double*)malloc(sizeof(double) * m);
  for (int j = 0; j < m; ++j) LW[j] = canon(c->logL[order[j]]);
  const double tau_e = LW[0];
  for (int j = 0; j < m; ++j)
    c->tau[j] = (c->cfg.correction == ORC_CORR_BEST_OF_WORST) ? LW[m - 1] : LW[j];
  /* seeds: uniform over the points ranked above W[j] */
  for (int j = 0; j < m; ++j) {
    double uu[2];
    orc_uniform2(c->cfg.seed, 0u, (uint32_t)j, (uint32_t)c->step, (uint32_t)ORC_STREAM_SEED << 24, uu);
    int r = j + 1 + (int)floor(uu[0] * (double)(N - j - 1));
    if (r > N - 1) r = N - 1;
    c->seeds[j] = order[r];
  }
  /* m independent chains */
  chain_stats* st = (chain_stats*)calloc(m, sizeof(chain_stats));
  double* hist_tmp = (double*)malloc(sizeof(double) * (long)T * m);
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 1)
  for (int j = 0; j < m; ++j) {
    double* hl = hist_tmp + (long)j * T;
    for (int t = 0; t < T; ++t) hl[t] = -INFINITY;
    slice_chain(c, j, c->seeds[j], c->tau[j], tau_e, c->new_u + (long)j * d, &c->new_logL[j],
                hl, c->hist_u + (long)j * T * d, &c->hist_n[j], &st[j], &c->brk[j]);
  }
  for (int j = 0; j < m; ++j) {
    for (int t = 0; t < T; ++t) c->hist_logL[(long)t * m + j] = hist_tmp[(long)j * T + t];
    c->chain_evals[j] = st[j].evals;
    c->evals += st[j].evals;
    c->oob += st[j].oob;
    c->so_caps += st[j].so_caps;
    c->sh_caps += st[j].sh_caps;
  }
  free(hist_tmp);
  free(st);

  /* correction */
  int *acc_code = (int*)malloc(sizeof(int) * m), *acc_h = (int*)malloc(sizeof(int) * m);
  int *rej_code = (int*)malloc(sizeof(int) * m), *rej_h = (int*)malloc(sizeof(int) * m);
  double *acc_l = (double*)malloc(sizeof(double) * m), *rej_l = (double*)malloc(sizeof(double) * m);
  orc_correct(m, c->cfg.correction, c->cfg.history_iters, T, LW, c->new_logL, c->tau,
              c->hist_logL, c->hist_n, acc_code, acc_h, acc_l, rej_code, rej_h, rej_l);

  /* point of an entry */
#define ENTRY_POINT(code, hs) \
  ((code) < m ? c->u + (long)order[(code)] * d \
              : ((hs) < 0 ? c->new_u + (long)((code) - m) * d \
                          : c->hist_u + ((long)((code) - m) * T + (hs)) * d))
  /* dead rows first (they may reference worst points that get overwritten) */
  double* dead_pts = (double*)malloc(sizeof(double) * m * d);
  for (int q = 0; q < m; ++q)
    memcpy(dead_pts + (long)q * d, ENTRY_POINT(rej_code[q], rej_h[q]), sizeof(double) * d);
  /* accepted new points into the slots of rejected worst points, in W order */
  int* rejw = (int*)malloc(sizeof(int) * m);
  int nrw = 0;
  for (int k = 0; k < m; ++k) {
    int dead = 0;
    for (int q = 0; q < m; ++q) if (rej_code[q] == k) { dead = 1; break; }
    if (dead) rejw[nrw++] = k;
  }
  int r = 0;
  for (int q = 0; q < m; ++q) {
    if (acc_code[q] < m) continue;
    int slot = order[rejw[r++]];
    memcpy(c->u + (long)slot * d, ENTRY_POINT(acc_code[q], acc_h[q]), sizeof(double) * d);
    c->logL[slot] = acc_l[q];
    c->label[slot] = orc_nearest_centre(&c->tree, c->u + (long)slot * d);
  }
#undef ENTRY_POINT
  for (int q = 0; q < m; ++q) dead_push(c, dead_pts + (long)q * d, rej_l[q]);
  c->since_cluster += m;
  c->step++;

  /* stopping rule: remaining evidence fraction */
  double mx = -INFINITY;
  for (int k = 0; k < N; ++k) if (c->logL[k] > mx) mx = c->logL[k];
  if (-(double)c->n_dead / (double)N + mx - c->logZ < log(c->cfg.stop_frac)) c->done = 1;

  free(dead_pts); free(rejw);
  free(acc_code); free(acc_h); free(rej_code); free(rej_h); free(acc_l); free(rej_l);
  free(order);
  free(LW);
  return c->done;
}

long orc_run(orc_ctx* c, int m, long max_steps) {
  long k = 0;
  while (k < max_steps && !c->done) {
    if (orc_step(c, m) < 0) break;
    ++k;
  }
  return k;
}

void orc_logZ(orc_ctx* c, double* logZ, double* sigma, double* H) {
  double lz = c->logZ, A = c->A;
  const double N = (double)c->N;
  const double base = -(double)c->n_dead / N - log(N);
  for (int k = 0; k < c->N; ++k) evid_add(&lz, &A, c->logL[k] + base, c->logL[k]);
  double h = A - lz;
  if (logZ) *logZ = lz;
  if (H) *H = h;
  if (sigma) *sigma = sqrt((h > 0.0 ? h : 0.0) / N);
}

long orc_n_dead(const orc_ctx* c) { return c->n_dead; }

void orc_get_dead(const orc_ctx* c, double* u, double* logL, double* logX, double* logw) {
  const double N = (double)c->N;
  const double lw0 = log(-expm1(-1.0 / N));
  for (long i = 0; i < c->n_dead; ++i) {
    if (u) memcpy(u + i * c->d, c->dead_u + i * c->d, sizeof(double) * c->d);
    if (logL) logL[i] = c->dead_logL[i];
    if (logX) logX[i] = -(double)(i + 1) / N;
    if (logw) logw[i] = (c->dead_logL[i] - (double)i / N) + lw0;
  }
}

void orc_get_live(const orc_ctx* c, double* u, double* logL, int* label) {
  if (u) memcpy(u, c->u, sizeof(double) * c->N * c->d);
  if (logL) memcpy(logL, c->logL, sizeof(double) * c->N);
  if (label) memcpy(label, c->label, sizeof(int) * c->N);
}

void orc_set_live(orc_ctx* c, const double* u, const double* logL, const int* label) {
  if (u) memcpy(c->u, u, sizeof(double) * c->N * c->d);
  if (logL) memcpy(c->logL, logL, sizeof(double) * c->N);
  if (label) memcpy(c->label, label, sizeof(int) * c->N);
}

void orc_get_tree(const orc_ctx* c, orc_tree* t) { *t = c->tree; }
void orc_set_tree(orc_ctx* c, const orc_tree* t) { c->tree = *t; }

void orc_get_counters(const orc_ctx* c, long* o) {
  o[0] = c->evals; o[1] = c->oob; o[2] = c->so_caps; o[3] = c->sh_caps;
  o[4] = c->step; o[5] = c->n_dead; o[6] = 0; o[7] = c->clusterings;
}

void orc_get_state(const orc_ctx* c, double* logZ_run, double* A_run, long* step, int* done) {
  if (logZ_run) *logZ_run = c->logZ;
  if (A_run) *A_run = c->A;
  if (step) *step = c->step;
  if (done) *done = c->done;
}

void orc_get_last_batch(const orc_ctx* c, int* seeds, double* tau, double* new_u, double* new_logL,
                        long* chain_evals, double* hist_logL, double* hist_u, int* hist_n) {
  const int m = c->last_m, d = c->d, T = c->cfg.hist_cap;
  if (seeds) memcpy(seeds, c->seeds, sizeof(int) * m);
  if (tau) memcpy(tau, c->tau, sizeof(double) * m);
  if (new_u) memcpy(new_u, c->new_u, sizeof(double) * m * d);
  if (new_logL) memcpy(new_logL, c->new_logL, sizeof(double) * m);
  if (chain_evals) memcpy(chain_evals, c->chain_evals, sizeof(long) * m);
  if (hist_logL) memcpy(hist_logL, c->hist_logL, sizeof(double) * (long)T * m);
  if (hist_u) memcpy(hist_u, c->hist_u, sizeof(double) * (long)T * m * d);
  if (hist_n) memcpy(hist_n, c->hist_n, sizeof(int) * m);
}

void orc_get_last_brackets(const orc_ctx* c, double* x0, double* v, double* a, double* b, int* ka, int* kb) {
  const int m = c->last_m, d = c->d;
  for (int j = 0; j < m; ++j) {
    const last_bracket* lb = &c->brk[j];
    if (x0) memcpy(x0 + (long)j * d, lb->x0, sizeof(double) * d);
    if (v) memcpy(v + (long)j * d, lb->v, sizeof(double) * d);
    if (a) a[j] = lb->a;
    if (b) b[j] = lb->b;
    if (ka) ka[j] = lb->ka;
    if (kb) kb[j] = lb->kb;
  }
}
