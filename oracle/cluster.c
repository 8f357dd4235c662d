/*
 * cluster.c -- cluster tree of the live points (Sec. 2.1).  TEST INFRASTRUCTURE.
 *
 * A binary tree of maximum depth D (heap indexed: root 0, children 2n+1 and
 * 2n+2) is filled by splitting every node with k-means, k = 2 (Lloyd).  Each
 * node gets its mean and unbiased covariance; the covariance is made positive
 * definite by clipping its eigenvalues from below (cyclic Jacobi eigen
 * decomposition) and is then Cholesky factorised.  The node volume is taken as
 * sqrt(det Sigma') = prod_i L_ii.  Pruning runs bottom-up: a node keeps its two
 * children only when both hold more than n_min points and their combined
 * (effective) volume is more than p*100 % below the node's own volume.  The
 * surviving leaves are the clusters; every live point is labelled with the
 * cluster on its path.  A point added between clusterings joins the cluster
 * whose centre is nearest.
 *
 * Readings where the paper is silent: deterministic farthest-point k-means
 * start, a point goes to the first centre on a distance tie, the clip floor is
 * eps * max(lambda_max, 1e-300) and the covariance is only rebuilt from the
 * clipped spectrum when some eigenvalue was actually raised.
 *
 * Pins: tests/test_oracle_select_cluster.py (brute-force optimal 2-partition
 * on tiny sets, reconstruction A = Q diag(l) Q^T, L L^T = Sigma',
 * rank-deficient input gets lambda_min = eps * lambda_max, separated blobs
 * split, one Gaussian and a uniform box do not) and tests/test_oracle_pins.py
 * (nearest accepted centre on a hand-built tree and during a run, lower node
 * id on a tie).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ns_oracle.h"

/* Cyclic Jacobi (Golub & Van Loan, Sec. 8.5): A = Q diag(evals) Q^T. */
int orc_jacobi_eig(int d, const double* A, double* evals, double* Q) {
  double* a = (double*)malloc(sizeof(double) * d * d);
  memcpy(a, A, sizeof(double) * d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) Q[i * d + j] = (i == j) ? 1.0 : 0.0;
  double frob = 0.0;
  for (int i = 0; i < d * d; ++i) frob += a[i] * a[i];
  int sweeps = 0;
  for (; sweeps < 60; ++sweeps) {
    double off = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q)
        if (p != q) off += a[p * d + q] * a[p * d + q];
    if (off <= 1e-30 * frob || off == 0.0) break;
    for (int p = 0; p < d - 1; ++p) {
      for (int q = p + 1; q < d; ++q) {
        double apq = a[p * d + q];
        if (apq == 0.0) continue;
        double app = a[p * d + p], aqq = a[q * d + q];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = t * c;
        /* A <- A J  (columns p, q) */
        for (int k = 0; k < d; ++k) {
          double akp = a[k * d + p], akq = a[k * d + q];
          a[k * d + p] = c * akp - s * akq;
          a[k * d + q] = s * akp + c * akq;
        }
        /* A <- J^T A  (rows p, q) */
        for (int k = 0; k < d; ++k) {
          double apk = a[p * d + k], aqk = a[q * d + k];
          a[p * d + k] = c * apk - s * aqk;
          a[q * d + k] = s * apk + c * aqk;
        }
        /* Q <- Q J */
        for (int k = 0; k < d; ++k) {
          double qkp = Q[k * d + p], qkq = Q[k * d + q];
          Q[k * d + p] = c * qkp - s * qkq;
          Q[k * d + q] = s * qkp + c * qkq;
        }
      }
    }
  }
  for (int i = 0; i < d; ++i) evals[i] = a[i * d + i];
  free(a);
  return sweeps;
}

/* Cholesky-Banachiewicz, row by row.  Returns 0 on success, -1 if not PD. */
int orc_cholesky(int d, const double* A, double* L) {
  for (int i = 0; i < d * d; ++i) L[i] = 0.0;
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = A[i * d + j];
      for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
      if (i == j) {
        if (!(s > 0.0)) return -1;
        L[i * d + i] = sqrt(s);
      } else {
        L[i * d + j] = s / L[j * d + j];
      }
    }
  }
  return 0;
}

double orc_regularise(int d, const double* cov, double eps, double* L, int* clipped) {
  double lam[ORC_MAXD];
  double* Q = (double*)malloc(sizeof(double) * d * d);
  double* S = (double*)malloc(sizeof(double) * d * d);
  orc_jacobi_eig(d, cov, lam, Q);
  double lmax = lam[0];
  for (int i = 1; i < d; ++i) if (lam[i] > lmax) lmax = lam[i];
  double floor_ = eps * (lmax > 1e-300 ? lmax : 1e-300);
  int clip = 0;
  for (int i = 0; i < d; ++i) if (lam[i] < floor_) { lam[i] = floor_; clip = 1; }
  if (clip) {
    for (int i = 0; i < d; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += Q[i * d + k] * lam[k] * Q[j * d + k];
        S[i * d + j] = s;
        S[j * d + i] = s;
      }
  } else {
    memcpy(S, cov, sizeof(double) * d * d);
  }
  if (orc_cholesky(d, S, L) != 0) {
    /* rounding pushed a clipped spectrum below zero: lift the diagonal once */
    for (int i = 0; i < d; ++i) S[i * d + i] += floor_;
    clip = 1;
    orc_cholesky(d, S, L);
  }
  double logV = 0.0;
  for (int i = 0; i < d; ++i) logV += log(L[i * d + i]);
  if (clipped) *clipped = clip;
  free(Q);
  free(S);
  return logV;
}

static double sqdist(int d, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) {
    double r = a[i] - b[i];
    s += r * r;
  }
  return s;
}

static double logaddexp2(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  double mx = a > b ? a : b;
  return mx + log1p(exp(-fabs(a - b)));
}

/* 2-means of the points idx[0..n-1]; side[k] = 0 (first centre) or 1.
 * ca_out / cb_out (may be NULL): the final centres. */
static void two_means(const double* u, int d, const int* idx, int n, int iters, int* side, double* ca_out,
                      double* cb_out) {
  double mu[ORC_MAXD] = {0}, ca[ORC_MAXD], cb[ORC_MAXD];
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < d; ++i) mu[i] += u[(long)idx[k] * d + i];
  for (int i = 0; i < d; ++i) mu[i] /= (double)n;
  int ia = 0;
  double best = -1.0;
  for (int k = 0; k < n; ++k) {
    double s = sqdist(d, u + (long)idx[k] * d, mu);
    if (s > best) { best = s; ia = k; }
  }
  int ib = 0;
  best = -1.0;
  for (int k = 0; k < n; ++k) {
    double s = sqdist(d, u + (long)idx[k] * d, u + (long)idx[ia] * d);
    if (s > best) { best = s; ib = k; }
  }
  memcpy(ca, u + (long)idx[ia] * d, sizeof(double) * d);
  memcpy(cb, u + (long)idx[ib] * d, sizeof(double) * d);
  for (int k = 0; k < n; ++k) {
    const double* x = u + (long)idx[k] * d;
    side[k] = sqdist(d, x, ca) <= sqdist(d, x, cb) ? 0 : 1;
  }
  for (int it = 0; it < iters; ++it) {
    double sa[ORC_MAXD] = {0}, sb[ORC_MAXD] = {0};
    int na = 0, nb = 0;
    for (int k = 0; k < n; ++k) {
      const double* x = u + (long)idx[k] * d;
      if (side[k] == 0) { for (int i = 0; i < d; ++i) sa[i] += x[i]; ++na; }
      else { for (int i = 0; i < d; ++i) sb[i] += x[i]; ++nb; }
    }
    if (na > 0) for (int i = 0; i < d; ++i) ca[i] = sa[i] / (double)na;
    if (nb > 0) for (int i = 0; i < d; ++i) cb[i] = sb[i] / (double)nb;
    int changed = 0;
    for (int k = 0; k < n; ++k) {
      const double* x = u + (long)idx[k] * d;
      int s = sqdist(d, x, ca) <= sqdist(d, x, cb) ? 0 : 1;
      if (s != side[k]) { side[k] = s; changed = 1; }
    }
    if (!changed) break;
  }
  if (ca_out) memcpy(ca_out, ca, sizeof(double) * d);
  if (cb_out) memcpy(cb_out, cb, sizeof(double) * d);
}

/* The split of one node holding all n points (Sec. 2.1): side per point and
 * the two centres, as the tree build computes them. */
void orc_two_means(const double* u, int n, int d, int iters, double* ca, double* cb, int* side) {
  int* idx = (int*)malloc(sizeof(int) * (size_t)n);
  for (int k = 0; k < n; ++k) idx[k] = k;
  two_means(u, d, idx, n, iters, side, ca, cb);
  free(idx);
}

static int level_of(int n) {
  int l = 0;
  while (n > 0) { n = (n - 1) / 2; ++l; }
  return l;
}

int orc_cluster(const double* u, int N, int d, int depth, double p, int nmin,
                int kmeans_iters, double eps, orc_tree* t, int* labels) {
  const int nodes = (1 << (depth + 1)) - 1;
  memset(t, 0, sizeof(*t));
  t->depth = depth;
  t->d = d;
  t->n_nodes = nodes;
  int* nodeof = (int*)malloc(sizeof(int) * N);
  int* idx = (int*)malloc(sizeof(int) * N);
  int* side = (int*)malloc(sizeof(int) * N);
  double* cov = (double*)malloc(sizeof(double) * d * d);
  for (int k = 0; k < N; ++k) nodeof[k] = 0;
  for (int n = 0; n < nodes; ++n) {
    int cnt = 0;
    for (int k = 0; k < N; ++k) if (nodeof[k] == n) idx[cnt++] = k;
    t->count[n] = cnt;
    double* c = t->centre + (long)n * ORC_MAXD;
    double* L = t->chol + (long)n * ORC_MAXD * ORC_MAXD;
    if (cnt >= 1) {
      for (int i = 0; i < d; ++i) c[i] = 0.0;
      for (int k = 0; k < cnt; ++k)
        for (int i = 0; i < d; ++i) c[i] += u[(long)idx[k] * d + i];
      for (int i = 0; i < d; ++i) c[i] /= (double)cnt;
    }
    if (cnt >= 2) {
      for (int i = 0; i < d; ++i)
        for (int j = 0; j <= i; ++j) {
          double s = 0.0;
          for (int k = 0; k < cnt; ++k) {
            const double* x = u + (long)idx[k] * d;
            s += (x[i] - c[i]) * (x[j] - c[j]);
          }
          s /= (double)(cnt - 1);
          cov[i * d + j] = s;
          cov[j * d + i] = s;
        }
      double Ld[ORC_MAXD * ORC_MAXD];
      t->logV[n] = orc_regularise(d, cov, eps, Ld, NULL);
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) L[i * ORC_MAXD + j] = Ld[i * d + j];
    } else {
      t->logV[n] = -INFINITY;
    }
    if (level_of(n) < depth && cnt >= 2) {
      two_means(u, d, idx, cnt, kmeans_iters, side, NULL, NULL);
      for (int k = 0; k < cnt; ++k) nodeof[idx[k]] = 2 * n + 1 + side[k];
    }
  }
  /* bottom-up pruning */
  const double logkeep = log(1.0 - p);
  for (int n = nodes - 1; n >= 0; --n) {
    t->split_ok[n] = 0;
    t->logV_eff[n] = t->logV[n];
    if (level_of(n) < depth) {
      int c1 = 2 * n + 1, c2 = 2 * n + 2;
      if (t->count[c1] > nmin && t->count[c2] > nmin) {
        double comb = logaddexp2(t->logV_eff[c1], t->logV_eff[c2]);
        if (comb < logkeep + t->logV[n]) {
          t->split_ok[n] = 1;
          t->logV_eff[n] = comb;
        }
      }
    }
  }
  /* accepted clusters: the cut reached from the root through kept splits */
  int reach[127];
  for (int n = 0; n < nodes; ++n) {
    reach[n] = (n == 0) ? 1 : (reach[(n - 1) / 2] && t->split_ok[(n - 1) / 2]);
    t->accepted[n] = reach[n] && !t->split_ok[n];
  }
  if (labels) {
    for (int k = 0; k < N; ++k) {
      int n = nodeof[k];
      while (!t->accepted[n]) n = (n - 1) / 2;
      labels[k] = n;
    }
  }
  free(nodeof);
  free(idx);
  free(side);
  free(cov);
  return 0;
}

int orc_nearest_centre(const orc_tree* t, const double* x) {
  int best = -1;
  double bd = INFINITY;
  for (int n = 0; n < t->n_nodes; ++n) {
    if (!t->accepted[n]) continue;
    double s = sqdist(t->d, x, t->centre + (long)n * ORC_MAXD);
    if (best < 0 || s < bd) { bd = s; best = n; }
  }
  return best;
}
