/*
 * mlp.c -- FP64 forward and backward of a fully connected network with a
 * linear output layer.  TEST INFRASTRUCTURE (oracle).
 *
 * Used for the emulator likelihood (tanh hidden layers) and for the learned
 * log-likelihood surrogate (SiLU hidden layers) trained on the sampler's own
 * (theta, logL) pairs.  Layout: X is B x widths[0] row major, W_l is
 * widths[l] x widths[l+1] row major, so layer l computes z = h W_l + b_l.
 * `acts` keeps every layer's pre-activation z (B x widths[l+1], layers
 * concatenated) for the backward pass.
 *
 * Pins: tests/test_oracle_mlp_quadrature.py checks the backward pass against
 * FP64 central finite differences of the forward pass;
 * tests/test_oracle_likelihood.py checks the forward pass against a plain
 * numpy matrix chain.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ns_oracle.h"

static double act_f(int act, double z) {
  if (act == 0) return tanh(z);
  return z / (1.0 + exp(-z));
}

static double act_df(int act, double z) {
  if (act == 0) {
    double t = tanh(z);
    return 1.0 - t * t;
  }
  double s = 1.0 / (1.0 + exp(-z));
  return s * (1.0 + z * (1.0 - s));
}

void orc_mlp_forward(int L, const int* w, const double* W, const double* b, int act,
                     const double* X, long B, double* Y, double* acts) {
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (w[l] > maxw) maxw = w[l];
  double* h = (double*)malloc(sizeof(double) * maxw);
  double* g = (double*)malloc(sizeof(double) * maxw);
  for (long r = 0; r < B; ++r) {
    for (int i = 0; i < w[0]; ++i) h[i] = X[r * w[0] + i];
    const double* Wl = W;
    const double* bl = b;
    long aoff = 0;
    for (int l = 0; l < L; ++l) {
      int nin = w[l], nout = w[l + 1];
      for (int j = 0; j < nout; ++j) {
        double s = 0.0;
        for (int i = 0; i < nin; ++i) s += h[i] * Wl[(long)i * nout + j];
        s += bl[j];
        if (acts) acts[aoff * B + r * nout + j] = s;
        g[j] = (l + 1 < L) ? act_f(act, s) : s;
      }
      aoff += nout;
      Wl += (long)nin * nout;
      bl += nout;
      double* t = h; h = g; g = t;
    }
    for (int j = 0; j < w[L]; ++j) Y[r * w[L] + j] = h[j];
  }
  free(h);
  free(g);
}

void orc_mlp_backward(int L, const int* w, const double* W, const double* b, int act,
                      const double* X, long B, const double* acts, const double* dY,
                      double* dW, double* db, double* dX) {
  (void)b;
  long nW = 0, nb = 0, na = 0;
  for (int l = 0; l < L; ++l) { nW += (long)w[l] * w[l + 1]; nb += w[l + 1]; na += w[l + 1]; }
  memset(dW, 0, sizeof(double) * nW);
  memset(db, 0, sizeof(double) * nb);
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (w[l] > maxw) maxw = w[l];
  double* delta = (double*)malloc(sizeof(double) * maxw);
  double* dh = (double*)malloc(sizeof(double) * maxw);
  double* hin = (double*)malloc(sizeof(double) * maxw);
  /* offsets of each layer's weights, biases and pre-activations */
  long* woff = (long*)malloc(sizeof(long) * (L + 1));
  long* boff = (long*)malloc(sizeof(long) * (L + 1));
  woff[0] = 0; boff[0] = 0;
  for (int l = 0; l < L; ++l) { woff[l + 1] = woff[l] + (long)w[l] * w[l + 1]; boff[l + 1] = boff[l] + w[l + 1]; }
  for (long r = 0; r < B; ++r) {
    for (int j = 0; j < w[L]; ++j) delta[j] = dY[r * w[L] + j];
    for (int l = L - 1; l >= 0; --l) {
      int nin = w[l], nout = w[l + 1];
      /* input of layer l */
      if (l == 0) {
        for (int i = 0; i < nin; ++i) hin[i] = X[r * nin + i];
      } else {
        const double* z = acts + boff[l - 1] * B + r * nin;
        for (int i = 0; i < nin; ++i) hin[i] = act_f(act, z[i]);
      }
      const double* Wl = W + woff[l];
      double* dWl = dW + woff[l];
      for (int i = 0; i < nin; ++i)
        for (int j = 0; j < nout; ++j) dWl[(long)i * nout + j] += hin[i] * delta[j];
      for (int j = 0; j < nout; ++j) db[boff[l] + j] += delta[j];
      for (int i = 0; i < nin; ++i) {
        double s = 0.0;
        for (int j = 0; j < nout; ++j) s += Wl[(long)i * nout + j] * delta[j];
        dh[i] = s;
      }
      if (l == 0) {
        if (dX) for (int i = 0; i < nin; ++i) dX[r * nin + i] = dh[i];
      } else {
        const double* z = acts + boff[l - 1] * B + r * nin;
        for (int i = 0; i < nin; ++i) delta[i] = dh[i] * act_df(act, z[i]);
      }
    }
  }
  (void)na;
  free(delta); free(dh); free(hin); free(woff); free(boff);
}
