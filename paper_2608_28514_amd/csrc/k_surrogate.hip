// k_surrogate.hip -- learned pre-screen of slice proposals and its online
// training on the (theta, logL) pairs the sampler evaluates.
//
// Per round of the batched slice sampler:
//   k_screen   : surrogate estimate logL_hat = mu + s * y_hat for every in-box
//                row; a row whose estimate lies below its threshold minus the
//                margin is screened out (treated as failing the constraint)
//                unless it is the audit_period-th screened row, which is still
//                evaluated; the rows to evaluate are compacted in order.
//   (emulator on the compacted rows)
//   k_scatter  : true logL back to the rows; audited rows that clear their
//                threshold count as false screens; every evaluated pair is
//                appended to the replay ring.
// Between steps, training: minibatches drawn (Philox) from the ring, targets
// max(logL, L_W[0] - floor_below) mapped to (t - mu)/s, MSE, the hand-written
// backward of k_gemm.hip, Adam.  Accepted points always carry their true logL.
#include "ns_internal.hpp"
#include "ns_gemm.hpp"
#include "ns_surrogate.hpp"

namespace ns {

constexpr int kST = 1024;

__device__ int scan_flag_s(int flag, int* wave_tot, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t bal = __ballot(flag);
  const int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wave_tot[wv] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int q = 0; q < nw; ++q) { const int v = wave_tot[q]; wave_tot[q] = acc; acc += v; }
    *total = acc;
  }
  __syncthreads();
  const int off = wave_tot[wv] + before;
  __syncthreads();
  return off;
}

__global__ void __launch_bounds__(kST)
k_screen(int M, int d, int screening, double margin, int audit_period, const int* __restrict__ flag,
         const double* __restrict__ rthr, const float* __restrict__ yhat, const float* __restrict__ norm,
         const float* __restrict__ xin, int* __restrict__ sflag, int* __restrict__ idx,
         int* __restrict__ aud, float* __restrict__ xc, int* __restrict__ count,
         double* __restrict__ rlogL, SurrCounters* __restrict__ sc, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int wave_tot[kST / 64];
  __shared__ int s_total;
  const float mu = norm[0], sd = norm[1];
  const unsigned long long sbase = sc->screened_seen;
  int n_eval = 0, n_scr = 0;
  for (int base = 0; base < M; base += kST) {
    const int r = base + threadIdx.x;
    const bool inb = r < M && flag[r] != 0;
    bool scr = false;
    if (inb && screening) {
      const double lhat = static_cast<double>(mu) + static_cast<double>(sd) * static_cast<double>(yhat[r]);
      scr = lhat < rthr[r] - margin;
    }
    // running index of screened rows decides the audits
    const int so = scan_flag_s(scr ? 1 : 0, wave_tot, &s_total);
    const int nscr_chunk = s_total;
    const bool audit = scr && ((sbase + n_scr + so) % static_cast<unsigned long long>(audit_period) == 0);
    const bool eval = inb && (!scr || audit);
    const int eo = scan_flag_s(eval ? 1 : 0, wave_tot, &s_total);
    if (r < M) {
      sflag[r] = (scr && !audit) ? 1 : 0;
      if (scr && !audit) rlogL[r] = -INFINITY;
      if (!inb) rlogL[r] = -INFINITY;
    }
    if (eval) {
      const int i = n_eval + eo;
      idx[i] = r;
      aud[i] = audit ? 1 : 0;
      for (int q = 0; q < d; ++q) xc[static_cast<long>(i) * d + q] = xin[static_cast<long>(r) * d + q];
    }
    n_eval += s_total;
    n_scr += nscr_chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *count = n_eval;
    sc->screened_seen = sbase + n_scr;
  }
}

hipError_t launch_screen(int M, int d, int screening, double margin, int audit_period, const int* flag,
                         const double* rthr, const float* yhat, const float* norm, const float* xin,
                         int* sflag, int* idx, int* aud, float* xc, int* count, double* rlogL,
                         SurrCounters* sc, const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_screen, dim3(1), dim3(kST), 0, s, M, d, screening, margin, audit_period, flag,
                     rthr, yhat, norm, xin, sflag, idx, aud, xc, count, rlogL, sc, gate);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kST)
k_scatter(int d, const int* __restrict__ count, const int* __restrict__ idx, const int* __restrict__ aud,
          const double* __restrict__ clogL, const double* __restrict__ rthr, const float* __restrict__ xc,
          double* __restrict__ rlogL, float* __restrict__ rep_x, double* __restrict__ rep_y, long cap,
          SurrCounters* __restrict__ sc, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int s_fn, s_aud;
  if (threadIdx.x == 0) { s_fn = 0; s_aud = 0; }
  __syncthreads();
  const int n = *count;
  const unsigned long long base = sc->pairs;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = idx[i];
    const double l = clogL[i];
    rlogL[r] = l;
    if (aud[i]) {
      atomicAdd(&s_aud, 1);
      if (l > rthr[r]) atomicAdd(&s_fn, 1);
    }
    if (cap > 0) {
      const long pos = static_cast<long>((base + i) % static_cast<unsigned long long>(cap));
      for (int q = 0; q < d; ++q) rep_x[pos * d + q] = xc[static_cast<long>(i) * d + q];
      rep_y[pos] = l;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // pairs counts the rows written to the ring (none before the ring exists),
    // so slots [0, min(pairs, cap)) always hold data
    if (cap > 0) sc->pairs = base + n;
    sc->emu_rows += n;
    sc->audited += s_aud;
    sc->false_screens += s_fn;
  }
}

hipError_t launch_scatter(int d, const int* count, const int* idx, const int* aud, const double* clogL,
                          const double* rthr, const float* xc, double* rlogL, float* rep_x, double* rep_y,
                          long cap, SurrCounters* sc, const int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(1), dim3(kST), 0, s, d, count, idx, aud, clogL, rthr, xc, rlogL, rep_x,
                     rep_y, cap, sc, gate);
  return hipGetLastError();
}

// Normalisation of the surrogate, refreshed at every training call:
//   output: t = max(logL, lo) mapped to (t - mu)/s, lo = L_W[0] - floor_below,
//           hi = max(best live logL, lo + floor_below), mu = (lo+hi)/2, s = (hi-lo)/2;
//   input:  theta standardised with the mean and standard deviation of the live
//           set (the root node of the cluster tree).
// norm = [mu, s, mean_0..mean_{d-1}, 1/std_0..1/std_{d-1}].
__global__ void k_sample_batch(int B, int d, uint64_t seed, uint32_t call, uint32_t iter,
                               const float* __restrict__ rep_x, const double* __restrict__ rep_y, long cap,
                               const SurrCounters* __restrict__ sc, const double* __restrict__ LW,
                               const RunState* __restrict__ st, const double* __restrict__ root_centre,
                               const double* __restrict__ root_cov, const double* __restrict__ lo_box,
                               const double* __restrict__ span_box, double floor_below,
                               float* __restrict__ Xb, float* __restrict__ yb, float* __restrict__ norm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long filled = sc->pairs < static_cast<unsigned long long>(cap)
                                        ? sc->pairs : static_cast<unsigned long long>(cap);
  const double lo = LW[0] - floor_below;
  const double hi = st->lmax > lo + floor_below ? st->lmax : lo + floor_below;
  const double mu = 0.5 * (lo + hi), s = 0.5 * (hi - lo);
  if (k == 0) { norm[0] = static_cast<float>(mu); norm[1] = static_cast<float>(s); }
  if (k < d) {
    // theta = lo + span u for the live set's unit-cube mean / covariance
    const double mean = lo_box[k] + span_box[k] * root_centre[k];
    const double var = span_box[k] * span_box[k] * root_cov[k * kMaxD + k];
    norm[2 + k] = static_cast<float>(mean);
    norm[2 + kMaxD + k] = static_cast<float>(1.0 / sqrt(var > 1e-30 ? var : 1e-30));
  }
  if (k >= B || filled == 0) return;
  const Draw2 u = uniform2(seed, static_cast<uint32_t>(k), call, iter, kStreamSurrogate << 24);
  long pos = static_cast<long>(floor(u.a * static_cast<double>(filled)));
  if (pos >= static_cast<long>(filled)) pos = static_cast<long>(filled) - 1;
  for (int q = 0; q < d; ++q) {
    const double mean = lo_box[q] + span_box[q] * root_centre[q];
    const double var = span_box[q] * span_box[q] * root_cov[q * kMaxD + q];
    const double istd = 1.0 / sqrt(var > 1e-30 ? var : 1e-30);
    Xb[static_cast<long>(k) * d + q] = static_cast<float>((rep_x[pos * d + q] - mean) * istd);
  }
  const double t = rep_y[pos] > lo ? rep_y[pos] : lo;
  yb[k] = static_cast<float>((t - mu) / s);
}

hipError_t launch_sample_batch(int B, int d, uint64_t seed, uint32_t call, uint32_t iter, const float* rep_x,
                               const double* rep_y, long cap, const SurrCounters* sc, const double* LW,
                               const RunState* st, const double* root_centre, const double* root_cov,
                               const double* lo_box, const double* span_box, double floor_below, float* Xb,
                               float* yb, float* norm, hipStream_t s) {
  const int n = B > d ? B : d;
  hipLaunchKernelGGL(k_sample_batch, dim3((n + 255) / 256), dim3(256), 0, s, B, d, seed, call, iter, rep_x,
                     rep_y, cap, sc, LW, st, root_centre, root_cov, lo_box, span_box, floor_below, Xb, yb,
                     norm);
  return hipGetLastError();
}

// Rows of network input theta -> standardised surrogate input (norm as above).
__global__ void k_standardize(long n, int d, const float* __restrict__ x, const float* __restrict__ norm,
                              float* __restrict__ xs, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int q = static_cast<int>(i % d);
  xs[i] = (x[i] - norm[2 + q]) * norm[2 + kMaxD + q];
}

hipError_t launch_standardize(long n, int d, const float* x, const float* norm, float* xs, const int* gate,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_standardize, dim3(static_cast<unsigned>((n * d + 255) / 256)), dim3(256), 0, s, n, d, x,
                     norm, xs, gate);
  return hipGetLastError();
}

// dY = 2 (yhat - y) / B and the mean squared error (one workgroup).
__global__ void __launch_bounds__(256)
k_mse_grad(int B, const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ dY,
           float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int k = threadIdx.x; k < B; k += blockDim.x) {
    const float e = yhat[k] - y[k];
    dY[k] = 2.f * e / static_cast<float>(B);
    s += e * e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / static_cast<float>(B);
}

hipError_t launch_mse_grad(int B, const float* yhat, const float* y, float* dY, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse_grad, dim3(1), dim3(256), 0, s, B, yhat, y, dY, loss);
  return hipGetLastError();
}

// Adam (Kingma & Ba) over a flat parameter vector; t = step number (1-based).
__global__ void k_adam(long n, float lr, float b1, float b2, float eps, int t, float* __restrict__ p,
                       const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, static_cast<float>(t)));
  const float vh = vi / (1.f - powf(b2, static_cast<float>(t)));
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_adam(long n, float lr, float b1, float b2, float eps, int t, float* p, const float* g,
                       float* m, float* v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, lr, b1, b2,
                     eps, t, p, g, m, v);
  return hipGetLastError();
}

// Glorot-uniform initialisation of a weight block from Philox (biases zero).
__global__ void k_glorot(long n, int fan_in, int fan_out, uint64_t seed, uint32_t layer, float* __restrict__ w) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Draw2 u = uniform2(seed, static_cast<uint32_t>(i), layer, 0xFFFFFFFFu, kStreamSurrogate << 24);
  const double a = sqrt(6.0 / static_cast<double>(fan_in + fan_out));
  w[i] = static_cast<float>((2.0 * u.a - 1.0) * a);
}

hipError_t launch_glorot(long n, int fan_in, int fan_out, uint64_t seed, uint32_t layer, float* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_glorot, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, fan_in,
                     fan_out, seed, layer, w);
  return hipGetLastError();
}

// logL_hat = mu + s * y_hat in place.
__global__ void k_norm_apply(long n, const float* __restrict__ norm, float* __restrict__ y) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = norm[0] + norm[1] * y[i];
}

hipError_t launch_norm_apply(long n, const float* norm, float* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm_apply, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, norm, y);
  return hipGetLastError();
}

}  // namespace ns
