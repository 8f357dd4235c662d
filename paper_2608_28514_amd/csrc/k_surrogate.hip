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
//                appended to the replay ring (k_scatter_final then advances
//                the counters).
// Between steps, training: minibatches drawn (Philox) from the ring, targets
// max(logL, L_W[0] - floor_below) mapped to (t - mu)/s, MSE, the hand-written
// backward of k_gemm.hip, Adam.  Accepted points always carry their true logL.
#include "ns_internal.hpp"
#include "ns_gemm.hpp"
#include "ns_surrogate.hpp"

namespace ns {


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

// Row screening and order-preserving compaction in two passes over chunks of
// kSC rows.  Pass 1 counts, per chunk, the in-box rows and the rows the
// surrogate places below threshold - margin.  Pass 2 gives every chunk its
// offsets: the screened rows before it (prefix of the counts), hence its
// audits in closed form (screened rows whose running index, counted from the
// rows screened in earlier calls, is a multiple of audit_period), hence the
// evaluated rows before it; then each chunk writes its rows in order.  The
// result is the one a single sequential pass gives.
constexpr int kSC = 256;

__device__ __forceinline__ bool screened_row(int r, int M, int screening, double margin, const int* flag,
                                             const double* rthr, const float* yhat, float mu, float sd,
                                             bool* inb) {
  *inb = r < M && flag[r] != 0;
  if (!*inb || !screening) return false;
  const double lhat = static_cast<double>(mu) + static_cast<double>(sd) * static_cast<double>(yhat[r]);
  return lhat < rthr[r] - margin;
}

// number of k in [a, a + n) with (base + k) % period == 0
__device__ __forceinline__ long long audits_in(unsigned long long base, long long a, long long n, long long period) {
  if (n <= 0) return 0;
  const unsigned long long lo = base + static_cast<unsigned long long>(a);
  const unsigned long long hi = lo + static_cast<unsigned long long>(n);   // exclusive
  const unsigned long long P = static_cast<unsigned long long>(period);
  return static_cast<long long>((hi + P - 1) / P - (lo + P - 1) / P);
}

__global__ void __launch_bounds__(kSC)
k_screen_count(int M, int screening, double margin, const int* __restrict__ flag,
               const double* __restrict__ rthr, const float* __restrict__ yhat,
               const float* __restrict__ norm, int* __restrict__ chunk_cnt, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int red[2 * (kSC / 64)];
  const int r = blockIdx.x * kSC + threadIdx.x;
  bool inb;
  const bool scr = screened_row(r, M, screening, margin, flag, rthr, yhat, norm[0], norm[1], &inb);
  const int ni = __popcll(__ballot(inb)), ns = __popcll(__ballot(scr));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { red[2 * wv] = ni; red[2 * wv + 1] = ns; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ti = 0, ts = 0;
    for (int q = 0; q < kSC / 64; ++q) { ti += red[2 * q]; ts += red[2 * q + 1]; }
    chunk_cnt[2 * blockIdx.x] = ti;
    chunk_cnt[2 * blockIdx.x + 1] = ts;
  }
}

__global__ void __launch_bounds__(kSC)
k_screen_write(int M, int d, int screening, double margin, int audit_period, const int* __restrict__ flag,
               const double* __restrict__ rthr, const float* __restrict__ yhat, const float* __restrict__ norm,
               const float* __restrict__ xin, const int* __restrict__ chunk_cnt, int* __restrict__ sflag,
               int* __restrict__ idx, int* __restrict__ aud, float* __restrict__ xc, __bf16* __restrict__ xf,
               long xfplane, int* __restrict__ count,
               double* __restrict__ rlogL, SurrCounters* __restrict__ sc, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int wave_tot[kSC / 64];
  __shared__ int s_total;
  __shared__ long long s_off[2];     // screened and evaluated rows before this chunk
  __shared__ int s_rows[kSC];
  const int nchunk = (M + kSC - 1) / kSC;
  const unsigned long long sbase = sc->screened_seen;
  const long long period = audit_period;
  if (threadIdx.x < 64) {
    // prefix over the chunks, 64 at a time (one lane each): screened rows
    // before each chunk, then the rows it evaluates (audits in closed form)
    const int lane = threadIdx.x;
    int carry_s = 0, carry_e = 0;
    for (int c0 = 0; c0 < nchunk; c0 += 64) {
      const int c = c0 + lane;
      const int ni = c < nchunk ? chunk_cnt[2 * c] : 0, ns = c < nchunk ? chunk_cnt[2 * c + 1] : 0;
      int is = ns;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(is, o);
        if (lane >= o) is += t;
      }
      const int ts = carry_s + is - ns;
      const int ev = c < nchunk ? (ni - ns) + static_cast<int>(audits_in(sbase, ts, ns, period)) : 0;
      int ie = ev;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(ie, o);
        if (lane >= o) ie += t;
      }
      if (c == static_cast<int>(blockIdx.x)) {
        s_off[0] = ts;
        s_off[1] = carry_e + ie - ev;
      }
      carry_s += __shfl(is, 63);
      carry_e += __shfl(ie, 63);
    }
    // count[0]: rows to evaluate; count[1]: rows screened by this call (added
    // to the running total by k_scatter, after every chunk has read it)
    if (blockIdx.x == 0 && lane == 0) {
      count[0] = carry_e;
      count[1] = carry_s;
    }
  }
  __syncthreads();
  const int r = blockIdx.x * kSC + threadIdx.x;
  bool inb;
  const bool scr = screened_row(r, M, screening, margin, flag, rthr, yhat, norm[0], norm[1], &inb);
  const int so = scan_flag_s(scr ? 1 : 0, wave_tot, &s_total);
  const bool audit = scr && ((sbase + static_cast<unsigned long long>(s_off[0] + so)) %
                             static_cast<unsigned long long>(period) == 0);
  const bool eval = inb && (!scr || audit);
  const int eo = scan_flag_s(eval ? 1 : 0, wave_tot, &s_total);
  const int n_eval = s_total;
  if (r < M) {
    sflag[r] = (scr && !audit) ? 1 : 0;
    if ((scr && !audit) || !inb) rlogL[r] = -INFINITY;
  }
  const long long base = s_off[1];
  if (eval) {
    idx[base + eo] = r;
    aud[base + eo] = audit ? 1 : 0;
    s_rows[eo] = r;
  }
  __syncthreads();
  // the chunk's evaluated rows, coordinates in order (consecutive threads read
  // consecutive coordinates of a row)
  // (eight loads in flight per thread before their stores)
  const int tot = n_eval * d;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * kSC) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = min(e0 + j * kSC, tot - 1), k = e / d;
      v[j] = xin[static_cast<long>(s_rows[k]) * d + (e - k * d)];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + j * kSC;
      if (e < tot) xc[base * d + e] = v[j];
    }
  }
  if (!xf) return;
  // the network input as three bfloat16 terms, fragment-major with 32 columns:
  // one item = 8 consecutive coordinates of a row (zero past d), 16-byte stores
  typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
  const int oct = (d + 7) >> 3, nit = n_eval * oct;
  for (int i0 = threadIdx.x; i0 < nit; i0 += 4 * kSC) {
    float v[4][8];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int it = min(i0 + a * kSC, nit - 1), k = it / oct, g = it - k * oct;
      const float* row = xin + static_cast<long>(s_rows[k]) * d;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[a][e] = row[min(8 * g + e, d - 1)];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int it = i0 + a * kSC;
      if (it >= nit) continue;
      const int k = it / oct, g = it - k * oct;
      bf16x8_t h, mm, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = 8 * g + e < d ? v[a][e] : 0.f;
        const __bf16 hh = static_cast<__bf16>(x);
        const float r1 = x - static_cast<float>(hh);
        const __bf16 m = static_cast<__bf16>(r1);
        h[e] = hh;
        mm[e] = m;
        lo[e] = static_cast<__bf16>(r1 - static_cast<float>(m));
      }
      const long fi = frag_index(base + k, 8 * g, 32);
      *reinterpret_cast<bf16x8_t*>(xf + fi) = h;
      *reinterpret_cast<bf16x8_t*>(xf + xfplane + fi) = mm;
      *reinterpret_cast<bf16x8_t*>(xf + 2 * xfplane + fi) = lo;
    }
  }
}

hipError_t launch_screen(int M, int d, int screening, double margin, int audit_period, const int* flag,
                         const double* rthr, const float* yhat, const float* norm, const float* xin,
                         int* sflag, int* idx, int* aud, float* xc, __bf16* xf, long xfplane, int* count,
                         double* rlogL, SurrCounters* sc, int* chunk_cnt, const int* gate, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int nchunk = (M + kSC - 1) / kSC;
  hipLaunchKernelGGL(k_screen_count, dim3(nchunk), dim3(kSC), 0, s, M, screening, margin, flag, rthr, yhat,
                     norm, chunk_cnt, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_screen_write, dim3(nchunk), dim3(kSC), 0, s, M, d, screening, margin, audit_period,
                     flag, rthr, yhat, norm, xin, chunk_cnt, sflag, idx, aud, xc, xf, xfplane, count, rlogL, sc,
                     gate);
  return hipGetLastError();
}

// True logL back to the rows, audits, and the replay-ring append, over
// chunks of 256 compacted rows (count[0] of them); every chunk reads the ring
// position sc->pairs, which k_scatter_final advances afterwards.
__global__ void __launch_bounds__(kSC)
k_scatter(int d, const int* __restrict__ count, const int* __restrict__ idx, const int* __restrict__ aud,
          const double* __restrict__ clogL, const double* __restrict__ part, int nb, long pstride,
          const double* __restrict__ rthr, const float* __restrict__ xc,
          double* __restrict__ rlogL, float* __restrict__ rep_x, double* __restrict__ rep_y, long cap,
          SurrCounters* __restrict__ sc, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int n = count[0];
  const int i0 = blockIdx.x * kSC;
  if (i0 >= n) return;
  const int i1 = min(n, i0 + kSC);
  __shared__ int s_fn, s_aud;
  if (threadIdx.x == 0) { s_fn = 0; s_aud = 0; }
  __syncthreads();
  const unsigned long long base = sc->pairs;
  const int i = i0 + threadIdx.x;
  if (i < i1) {
    const int r = idx[i];
    double l;
    if (part) {
      // chi^2 column-block partials of compacted row i, summed in block order
      double t = 0.0;
      for (int q0 = 0; q0 < nb; q0 += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = part[min(q0 + j, nb - 1) * pstride + i];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (q0 + j < nb) t += v[j];
      }
      const double v = -0.5 * t;
      l = isnan(v) ? -INFINITY : v;
    } else {
      l = clogL[i];
    }
    rlogL[r] = l;
    if (aud[i]) {
      atomicAdd(&s_aud, 1);
      if (l > rthr[r]) atomicAdd(&s_fn, 1);
    }
    if (cap > 0) rep_y[static_cast<long>((base + i) % static_cast<unsigned long long>(cap))] = l;
  }
  if (cap > 0) {
    const int tot = (i1 - i0) * d;
    for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * kSC) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = xc[static_cast<long>(i0) * d + min(e0 + j * kSC, tot - 1)];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = e0 + j * kSC;
        if (e >= tot) continue;
        const int k = e / d, q = e - k * d;
        const long pos = static_cast<long>((base + i0 + k) % static_cast<unsigned long long>(cap));
        rep_x[pos * d + q] = v[j];
      }
    }
  }
  __syncthreads();
  // integer counts: the same totals whatever the order of the chunks
  if (threadIdx.x == 0 && s_aud) atomicAdd(&sc->audited, static_cast<unsigned long long>(s_aud));
  if (threadIdx.x == 0 && s_fn) atomicAdd(&sc->false_screens, static_cast<unsigned long long>(s_fn));
}

__global__ void k_scatter_final(const int* __restrict__ count, long cap, SurrCounters* __restrict__ sc,
                                const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  if (threadIdx.x != 0) return;
  const int n = count[0];
  sc->screened_seen += static_cast<unsigned long long>(count[1]);
  // pairs counts the rows written to the ring (none before the ring exists),
  // so slots [0, min(pairs, cap)) always hold data
  if (cap > 0) sc->pairs += static_cast<unsigned long long>(n);
  sc->emu_rows += static_cast<unsigned long long>(n);
}

hipError_t launch_scatter(int M, int d, const int* count, const int* idx, const int* aud, const double* clogL,
                          const double* part, int nb, const double* rthr, const float* xc, double* rlogL,
                          float* rep_x, double* rep_y, long cap, SurrCounters* sc, const int* gate,
                          hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((M + kSC - 1) / kSC), dim3(kSC), 0, s, d, count, idx, aud, clogL, part, nb,
                     static_cast<long>(M), rthr, xc, rlogL, rep_x, rep_y, cap, sc, gate);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_final, dim3(1), dim3(64), 0, s, count, cap, sc, gate);
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
