/*
 * likelihood.c -- FP64 log-likelihoods of the oracle.  TEST INFRASTRUCTURE.
 *
 * The prior is uniform on the box [lo, hi]; points are carried in unit-cube
 * coordinates u and mapped to theta = lo + (hi - lo) u.  A point outside the
 * box has zero prior mass and is given logL = -inf; a NaN likelihood is also
 * mapped to -inf so that it can never satisfy a hard constraint.
 *
 *  - mixture: logL = log sum_k w_k exp(-q_k / 2), q_k a diagonal Mahalanobis
 *    distance.  Covers the normalised Gaussian, the 4-Gaussian mixture, the
 *    Gaussian of Eq. (5), the 49-Gaussian array of Eq. (2) and the two
 *    separated Gaussians of Eq. (3).
 *  - Rosenbrock chain, Eq. (6) generalised to d dimensions.
 *  - Gaussian shell, Eq. (4).
 *  - MLP emulator: tanh hidden layers, linear output, diagonal chi^2 against a
 *    data vector (stands in for the emulated likelihood of Sec. 5).
 *
 * Pins (tests/test_oracle_likelihood.py): values at the mode and other special
 * points, closed-form evidences by quadrature, and the MLP against a plain
 * matrix product written independently with numpy.
 */
#include <math.h>
#include <stdlib.h>
#include <omp.h>
#include "ns_oracle.h"

static double lik_mixture(const orc_lik* L, const double* th) {
  const int d = L->d, K = L->n_comp;
  if (K == 1) {
    double q = 0.0;
    for (int i = 0; i < d; ++i) {
      double r = th[i] - L->mu[i];
      q += r * r * L->ivar[i];
    }
    return L->logw[0] - 0.5 * q;
  }
  double best = -INFINITY;
  double e[256];
  for (int k = 0; k < K && k < 256; ++k) {
    double q = 0.0;
    for (int i = 0; i < d; ++i) {
      double r = th[i] - L->mu[k * d + i];
      q += r * r * L->ivar[k * d + i];
    }
    e[k] = L->logw[k] - 0.5 * q;
    if (e[k] > best) best = e[k];
  }
  if (best == -INFINITY) return -INFINITY;
  double s = 0.0;
  for (int k = 0; k < K && k < 256; ++k) s += exp(e[k] - best);
  return best + log(s);
}

static double lik_rosenbrock(const orc_lik* L, const double* th) {
  double s = 0.0;
  for (int i = 0; i + 1 < L->d; ++i) {
    double t = th[i + 1] - th[i] * th[i];
    double r = L->ros_a - th[i];
    s += L->ros_b * t * t + r * r;
  }
  return -s;
}

static double lik_shell(const orc_lik* L, const double* th) {
  double s = 0.0;
  for (int i = 0; i < L->d; ++i) s += th[i] * th[i];
  double r = (sqrt(s) - L->shell_r0) / L->shell_w;
  return -0.5 * r * r;
}

/* Layer l: z_j = (sum_i a_i W_ij) + b_j, the sum over inputs i in ascending
 * order for every output j.  The loop runs over inputs on the outside and
 * outputs inside (one accumulator per output), so W is read row by row. */
static double lik_mlp(const orc_lik* L, const double* th) {
  int maxw = 0;
  for (int l = 0; l <= L->n_layers; ++l) if (L->widths[l] > maxw) maxw = L->widths[l];
  double* a = (double*)malloc(sizeof(double) * maxw);
  double* b = (double*)malloc(sizeof(double) * maxw);
  for (int i = 0; i < L->widths[0]; ++i) a[i] = th[i];
  const double* W = L->weights;
  const double* bias = L->biases;
  for (int l = 0; l < L->n_layers; ++l) {
    int nin = L->widths[l], nout = L->widths[l + 1];
    for (int j = 0; j < nout; ++j) b[j] = 0.0;
    for (int i = 0; i < nin; ++i) {
      const double ai = a[i];
      const double* Wi = W + (long)i * nout;
      for (int j = 0; j < nout; ++j) b[j] += ai * Wi[j];
    }
    for (int j = 0; j < nout; ++j) {
      double s = b[j] + bias[j];
      b[j] = (l + 1 < L->n_layers) ? tanh(s) : s;
    }
    W += (long)nin * nout;
    bias += nout;
    double* t = a; a = b; b = t;
  }
  int nout = L->widths[L->n_layers];
  double chi2 = 0.0;
  for (int i = 0; i < nout; ++i) {
    double r = (a[i] - L->data[i]) / L->sigma[i];
    chi2 += r * r;
  }
  free(a);
  free(b);
  return -0.5 * chi2;
}

static double loglike_one(const orc_lik* L, const double* th) {
  switch (L->kind) {
    case ORC_LIK_MIXTURE: return lik_mixture(L, th);
    case ORC_LIK_ROSENBROCK: return lik_rosenbrock(L, th);
    case ORC_LIK_SHELL: return lik_shell(L, th);
    case ORC_LIK_MLP: return lik_mlp(L, th);
    default: return NAN;
  }
}

void orc_loglike(const orc_lik* L, const double* lo, const double* hi,
                 const double* u, long n, double* out) {
  const int d = L->d;
  /* points are independent: spread them over the oracle's threads when not
     already inside a parallel region (the chains of a step) */
#pragma omp parallel for num_threads(orc_get_threads()) schedule(dynamic, 16) if (n > 1 && !omp_in_parallel())
  for (long k = 0; k < n; ++k) {
    double th[ORC_MAXD];
    const double* x = u + k * d;
    int inbox = 1;
    for (int i = 0; i < d; ++i) {
      if (!(x[i] >= 0.0 && x[i] <= 1.0)) inbox = 0;
      th[i] = lo[i] + (hi[i] - lo[i]) * x[i];
    }
    if (!inbox) { out[k] = -INFINITY; continue; }
    double v = loglike_one(L, th);
    out[k] = isnan(v) ? -INFINITY : v;
  }
}
