// k_select.hip -- selection of the m worst live points and the chains' seeds
// (Algorithm 1: "sorted", S_W, W, RNG.choose), plus the initial live points
// (uniform draws in the prior box) and the stand-alone likelihood / generator
// kernels.
//
// The whole live set (N <= 8192 keys) is sorted by one workgroup in LDS with a
// bitonic network on the composite key (order-preserving FP64 bits, slot), so
// the order is unique and identical to a stable sort on (logL, slot).
#include "ns_internal.hpp"
#include "ns_sort.hpp"

namespace ns {

constexpr int kSortMax = 8192;
constexpr int kSortThreads = 1024;


// Sort the first N entries of (keys, slots) in LDS; P = power of two >= N.
__device__ void bitonic_sort_lds(uint64_t* keys, int* slots, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const uint64_t ka = keys[i], kb = keys[ixj];
          const int sa = slots[i], sb = slots[ixj];
          const bool gt = key_less(kb, sb, ka, sa);
          if (gt == up) {
            keys[i] = kb; keys[ixj] = ka;
            slots[i] = sb; slots[ixj] = sa;
          }
        }
      }
      __syncthreads();
    }
  }
}


// Threads per sorting workgroup for N keys.
__host__ __device__ inline int sort_threads(int N) {
  const int P = sort_width(N);
  return P <= kSmallSort ? P / 2 : kSortThreads;
}

__device__ void sort_order(const double* __restrict__ logL, int N, int* __restrict__ order,
                           uint64_t* keys, int* slots) {
  const int P = sort_width(N);
  if (P <= kSmallSort) {
    sort_small(LogLKey{logL, N}, P, keys, slots);
  } else {
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
      if (i < N) { keys[i] = order_key(logL[i]); slots[i] = i; }
      else { keys[i] = ~0ull; slots[i] = 0x7fffffff; }
    }
    __syncthreads();
    bitonic_sort_lds(keys, slots, P);
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) order[i] = slots[i];
  __syncthreads();
}

__global__ void __launch_bounds__(kSortThreads)
k_select(const double* __restrict__ logL, int N, int m, int corr, uint64_t seed,
         int* __restrict__ order, double* __restrict__ LW, double* __restrict__ tau,
         int* __restrict__ seeds, const RunState* __restrict__ st) {
  if (st->done) return;
  __shared__ uint64_t keys[kSortMax];
  __shared__ int slots[kSortMax];
  sort_order(logL, N, order, keys, slots);
  const uint32_t step = static_cast<uint32_t>(st->step);
  const double lw_last = canon(logL[slots[m - 1]]);
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const double lw = canon(logL[slots[j]]);
    LW[j] = lw;
    tau[j] = (corr == kBestOfWorst) ? lw_last : lw;
    const Draw2 u = uniform2(seed, 0u, static_cast<uint32_t>(j), step, kStreamSeed << 24);
    int r = j + 1 + static_cast<int>(floor(u.a * static_cast<double>(N - j - 1)));
    if (r > N - 1) r = N - 1;
    seeds[j] = slots[r];
  }
}

__global__ void __launch_bounds__(kSortThreads)
k_select_order(const double* __restrict__ logL, int N, int* __restrict__ order) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int slots[kSortMax];
  sort_order(logL, N, order, keys, slots);
}

hipError_t launch_select(const Shape& sh, const DevBufs& b, int m, int corr, uint64_t seed,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(sort_threads(sh.N)), 0, s, b.logL, sh.N, m, corr, seed,
                     b.order, b.LW, b.tau, b.seeds, b.st);
  return hipGetLastError();
}

hipError_t launch_select_order(const double* logL, int N, int* order, hipStream_t s) {
  hipLaunchKernelGGL(k_select_order, dim3(1), dim3(sort_threads(N)), 0, s, logL, N, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial live points: u_k drawn uniformly in the unit cube, then logL.
template <typename T, typename LT>
__global__ void k_init_points(int N, int d, uint64_t seed, LikDev lik, T* __restrict__ u,
                              double* __restrict__ logL, RunState* __restrict__ st) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  T* y = u + static_cast<long>(k) * d;
  for (int p = 0; 2 * p < d; ++p) {
    const Draw2 w = uniform2(seed, static_cast<uint32_t>(p), static_cast<uint32_t>(k), 0u,
                             kStreamInit << 24);
    y[2 * p] = static_cast<T>(w.a);
    if (2 * p + 1 < d) y[2 * p + 1] = static_cast<T>(w.b);
  }
  double v = in_box(y, d) ? LikAt<LT>::eval(lik, PtAt<T>{y}) : -INFINITY;
  if (isnan(v)) atomicAdd(&st->nan_logL, 1ull);
  logL[k] = clean_logL(v);
}

hipError_t launch_init_points(const Shape& sh, const DevBufs& b, const LikDev& lik, uint64_t seed,
                              hipStream_t s) {
  const dim3 grid((sh.N + 255) / 256), block(256);
  if (sh.state_f32) {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_init_points<float, float>), grid, block, 0, s, sh.N, sh.d, seed, lik,
                         static_cast<float*>(b.u), b.logL, b.st);
    else
      hipLaunchKernelGGL((k_init_points<float, double>), grid, block, 0, s, sh.N, sh.d, seed, lik,
                         static_cast<float*>(b.u), b.logL, b.st);
  } else {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_init_points<double, float>), grid, block, 0, s, sh.N, sh.d, seed, lik,
                         static_cast<double*>(b.u), b.logL, b.st);
    else
      hipLaunchKernelGGL((k_init_points<double, double>), grid, block, 0, s, sh.N, sh.d, seed, lik,
                         static_cast<double*>(b.u), b.logL, b.st);
  }
  return hipGetLastError();
}

// Likelihood of arbitrary unit-cube points, rounded to the state precision
// exactly as the sampler stores them.
template <typename T>
struct CvtAt {
  const double* p;
  __device__ T operator()(int i) const { return static_cast<T>(p[i]); }
};

template <typename T, typename LT>
__global__ void k_loglike_points(int d, LikDev lik, const double* __restrict__ u, long n,
                                 double* __restrict__ out) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const CvtAt<T> y{u + k * d};
  bool ok = true;
  for (int i = 0; i < d; ++i) {
    const T yi = y(i);
    ok &= (yi >= T(0)) & (yi <= T(1));
  }
  out[k] = ok ? clean_logL(LikAt<LT>::eval(lik, y)) : -INFINITY;
}

hipError_t launch_loglike_points(const Shape& sh, const LikDev& lik, const double* u, long n,
                                 double* out, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  if (n == 0) return hipSuccess;
  if (sh.state_f32) {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_loglike_points<float, float>), grid, block, 0, s, sh.d, lik, u, n, out);
    else
      hipLaunchKernelGGL((k_loglike_points<float, double>), grid, block, 0, s, sh.d, lik, u, n, out);
  } else {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_loglike_points<double, float>), grid, block, 0, s, sh.d, lik, u, n, out);
    else
      hipLaunchKernelGGL((k_loglike_points<double, double>), grid, block, 0, s, sh.d, lik, u, n, out);
  }
  return hipGetLastError();
}

__global__ void k_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, long n,
                         uint32_t* __restrict__ out) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const U4 w = philox4x32_10(U4{c0 + static_cast<uint32_t>(k), c1, c2, c3},
                             static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  out[4 * k + 0] = w.x;
  out[4 * k + 1] = w.y;
  out[4 * k + 2] = w.z;
  out[4 * k + 3] = w.w;
}

hipError_t launch_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, long n,
                         uint32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, seed,
                     c0, c1, c2, c3, n, out);
  return hipGetLastError();
}

}  // namespace ns
