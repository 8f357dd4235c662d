// k_cluster_large.hip -- one node of the cluster tree (Sec. 2.1) for point
// sets far beyond one workgroup: mean, unbiased covariance and the k-means
// split (k = 2, Lloyd) of N points, as the tree kernels compute them per node.
//
// Every statistic is one streaming pass over the points: workgroups of one
// wave take contiguous chunks, each lane accumulates its points in FP64, the
// wave reduces with a fixed butterfly and writes one partial per workgroup; a
// single workgroup then adds the partials in workgroup order (deterministic).
// The split starts from the point farthest from the mean and the point
// farthest from that one (lowest index on ties), assigns a point to the first
// centre on a distance tie, and runs Lloyd updates until no assignment
// changes or after `iters` updates; an empty side keeps its centre.  Passes
// after the stop exit at once.
#include <algorithm>
#include "ns_device.hpp"
#include "ns_cluster_large.hpp"

namespace ns {

constexpr int kCLGroups = 2048;     // workgroups (one wave each) of a pass
constexpr int kCLPart = 528;        // doubles per partial: max(d (d + 1) / 2, 2 d + 2) for d <= 32

struct CLState {
  double ca[kMaxD], cb[kMaxD];
  int ia, ib;
  int done, passes, iters_used;
  int n0, n1;
};

struct CLWork {
  CLState st;
  double pad[8];
  double part[kCLGroups][kCLPart];
  double pv[kCLGroups];
  long pi[kCLGroups];
};

size_t cluster_split_work_bytes() { return sizeof(CLWork); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// chunk of workgroup g: points [lo, hi)
__device__ __forceinline__ void chunk_of(long N, long* lo, long* hi) {
  const long per = (N + gridDim.x - 1) / gridDim.x;
  *lo = min(N, static_cast<long>(blockIdx.x) * per);
  *hi = min(N, *lo + per);
}

template <int DM>
__device__ __forceinline__ double sqdist_pt(const float* x, const double* c, int d) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double q = static_cast<double>(x[i]) - c[i];
      s += q * q;
    }
  return s;
}


// Sum over the G partials of columns [c0, c0 + nc) (nc <= 32) by 256 threads:
// thread t adds partials t, t + 256, ... (eight loads in flight), then a
// fixed binary tree over the 256 threads.  out (LDS): out[c] for c < nc.
__device__ void sum_partials(const CLWork* w, int groups, int c0, int nc, double* red /* 256 x 33 */,
                             double* out) {
  const int t = threadIdx.x;
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int g0 = t; g0 < groups; g0 += 8 * 256) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int g = g0 + 256 * j;
      if (g >= groups) break;
      const double* row = w->part[g] + c0;
#pragma unroll
      for (int c = 0; c < 32; ++c)
        if (c < nc) acc[c] += row[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 32; ++c)
    if (c < nc) red[t * 33 + c] = acc[c];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
      for (int c = 0; c < nc; ++c) red[t * 33 + c] += red[(t + off) * 33 + c];
    __syncthreads();
  }
  if (t < nc) out[t] = red[t];
  __syncthreads();
}

// pass: coordinate sums (mean).  DM: the dimension rounded up to 2, 4, 8, 16 or 32.
template <int DM>
__global__ void __launch_bounds__(64) k_cl_sum(const float* __restrict__ u, long N, int d, CLWork* __restrict__ w) {
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x;
  double s[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) s[i] = 0.0;
  for (long k0 = lo + lane; k0 < hi; k0 += 4 * 64) {
    // four points' coordinates loaded before they are added (in point order)
    float xv[4][DM];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long k = min(k0 + 64 * j, hi - 1);
#pragma unroll
      for (int i = 0; i < DM; ++i) xv[j][i] = i < d ? u[k * d + i] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (k0 + 64 * j < hi)
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) s[i] += static_cast<double>(xv[j][i]);
  }
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double t = wave_sum(s[i]);
      if (lane == 0) w->part[blockIdx.x][i] = t;
    }
}

__global__ void __launch_bounds__(256)
k_cl_mean(long N, int d, int groups, double* __restrict__ mean, CLWork* __restrict__ w) {
  __shared__ double red[256 * 33];
  __shared__ double tot[32];
  sum_partials(w, groups, 0, d, red, tot);
  const int i = threadIdx.x;
  if (i < d) mean[i] = tot[i] / static_cast<double>(N);
  if (i == 0) {
    w->st.done = 0;
    w->st.passes = 1;
    w->st.iters_used = 0;
  }
}

// pass: centred outer products (lower triangle, row by row), d <= 12: every
// lane keeps the whole triangle of its points in registers, then the wave
// reduces each entry with the fixed butterfly
template <int DM>
__global__ void __launch_bounds__(64)
k_cl_cov_reg(const float* __restrict__ u, long N, int d, const double* __restrict__ mean, CLWork* __restrict__ w) {
  constexpr int NP = DM * (DM + 1) / 2;
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x;
  double mu[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) mu[i] = i < d ? mean[i] : 0.0;
  double acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.0;
  for (long k0 = lo + lane; k0 < hi; k0 += 2 * 64) {
    float xv[2][DM];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long k = min(k0 + 64 * j, hi - 1);
#pragma unroll
      for (int i = 0; i < DM; ++i) xv[j][i] = i < d ? u[k * d + i] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (k0 + 64 * j >= hi) continue;
      double x[DM];
#pragma unroll
      for (int i = 0; i < DM; ++i) x[i] = static_cast<double>(xv[j][i]) - mu[i];
      int p = 0;
#pragma unroll
      for (int i = 0; i < DM; ++i)
#pragma unroll
        for (int jj = 0; jj <= i; ++jj, ++p)
          if (i < d) acc[p] += x[i] * x[jj];
    }
  }
  // entry (i, jj) of the DM triangle is entry i (i + 1) / 2 + jj of the d triangle too
  int p = 0;
#pragma unroll
  for (int i = 0; i < DM; ++i)
#pragma unroll
    for (int jj = 0; jj <= i; ++jj, ++p)
      if (i < d) {
        const double t = wave_sum(acc[p]);
        if (lane == 0) w->part[blockIdx.x][p] = t;
      }
}

// pass: centred outer products (lower triangle, row by row), any d <= 32:
// points staged in LDS, lanes own entries
__global__ void __launch_bounds__(64)
k_cl_cov(const float* __restrict__ u, long N, int d, const double* __restrict__ mean, CLWork* __restrict__ w) {
  __shared__ double xs[64][kMaxD + 1];
  __shared__ double mu[kMaxD];
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x;
  if (lane < d) mu[lane] = mean[lane];
  const int np = d * (d + 1) / 2;
  // lane owns pairs lane, lane + 64, ... (at most 9 for d = 32)
  double acc[9];
  int pi_[9], pj_[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    acc[q] = 0.0;
    int p = lane + 64 * q, ii = 0;
    if (p < np) {
      while (p > ii) { p -= ii + 1; ++ii; }
    }
    pi_[q] = ii;
    pj_[q] = p;
  }
  __syncthreads();
  for (long k0 = lo; k0 < hi; k0 += 64) {
    const long k = k0 + lane;
    if (k < hi) {
#pragma unroll
      for (int i = 0; i < kMaxD; ++i)
        if (i < d) xs[lane][i] = static_cast<double>(u[k * d + i]) - mu[i];
    }
    __syncthreads();
    const int n = static_cast<int>(min(64L, hi - k0));
    for (int r = 0; r < n; ++r)
#pragma unroll
      for (int q = 0; q < 9; ++q)
        if (lane + 64 * q < np) acc[q] += xs[r][pi_[q]] * xs[r][pj_[q]];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 9; ++q)
    if (lane + 64 * q < np) w->part[blockIdx.x][lane + 64 * q] = acc[q];
}

// one workgroup per block of 32 pairs
__global__ void __launch_bounds__(256)
k_cl_covred(long N, int d, int groups, double* __restrict__ cov, CLWork* __restrict__ w) {
  __shared__ double red[256 * 33];
  const int np = d * (d + 1) / 2;
  const int c0 = blockIdx.x * 32, nc = min(32, np - c0);
  __shared__ double tot[32];
  sum_partials(w, groups, c0, nc, red, tot);
  const int q = threadIdx.x;
  if (q < nc) {
    int ii = 0, jj = c0 + q;
    while (jj > ii) { jj -= ii + 1; ++ii; }
    const double v = tot[q] / static_cast<double>(N - 1);
    cov[ii * d + jj] = v;
    cov[jj * d + ii] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w->st.passes += 1;
}

// pass: farthest point from ref (which = 0: the mean, 1: point ia), lowest index on ties
template <int DM>
__global__ void __launch_bounds__(64)
k_cl_far(const float* __restrict__ u, long N, int d, int which, const double* __restrict__ mean,
         CLWork* __restrict__ w) {
  __shared__ double ref[kMaxD];
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x;
  if (lane < d) ref[lane] = which == 0 ? mean[lane] : static_cast<double>(u[static_cast<long>(w->st.ia) * d + lane]);
  __syncthreads();
  double bv = -1.0;
  long bi = 0x7fffffffffffffffL;
  for (long k0 = lo + lane; k0 < hi; k0 += 4 * 64) {
    float xv[4][DM];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long k = min(k0 + 64 * j, hi - 1);
#pragma unroll
      for (int i = 0; i < DM; ++i) xv[j][i] = i < d ? u[k * d + i] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long k = k0 + 64 * j;
      if (k >= hi) continue;
      const double s = sqdist_pt<DM>(xv[j], ref, d);
      if (s > bv) { bv = s; bi = k; }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const long oi = __shfl_xor(bi, o);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) {
    w->pv[blockIdx.x] = bv;
    w->pi[blockIdx.x] = bi;
  }
}

__global__ void __launch_bounds__(256)
k_cl_farred(const float* __restrict__ u, int d, int groups, int which, CLWork* __restrict__ w) {
  __shared__ long s_i;
  __shared__ double sv[256];
  __shared__ long si[256];
  const int t = threadIdx.x;
  double bv = -1.0;
  long bi = 0x7fffffffffffffffL;
  for (int g0 = t; g0 < groups; g0 += 8 * 256) {
    double v[8];
    long ix[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int g = min(g0 + 256 * j, groups - 1);
      v[j] = w->pv[g];
      ix[j] = w->pi[g];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (g0 + 256 * j < groups && (v[j] > bv || (v[j] == bv && ix[j] < bi))) { bv = v[j]; bi = ix[j]; }
  }
  sv[t] = bv;
  si[t] = bi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off && (sv[t + off] > sv[t] || (sv[t + off] == sv[t] && si[t + off] < si[t]))) {
      sv[t] = sv[t + off];
      si[t] = si[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    s_i = si[0];
    if (which == 0) w->st.ia = static_cast<int>(si[0]); else w->st.ib = static_cast<int>(si[0]);
    w->st.passes += 1;
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < d) {
    const double v = static_cast<double>(u[s_i * d + i]);
    if (which == 0) w->st.ca[i] = v; else w->st.cb[i] = v;
  }
}

// Lloyd pass r: assign with the current centres (pass 0: the start pair),
// note changes, and sum the coordinates of each side
template <int DM>
__global__ void __launch_bounds__(64)
k_cl_lloyd(const float* __restrict__ u, long N, int d, int r, unsigned char* __restrict__ side,
           CLWork* __restrict__ w) {
  __shared__ double ca[kMaxD], cb[kMaxD];
  if (w->st.done) return;
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x;
  if (lane < d) { ca[lane] = w->st.ca[lane]; cb[lane] = w->st.cb[lane]; }
  __syncthreads();
  double sa[DM], sb[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) { sa[i] = 0.0; sb[i] = 0.0; }
  int n1 = 0, ch = 0;
  for (long k0 = lo + lane; k0 < hi; k0 += 2 * 64) {
    // two points' coordinates and previous sides loaded together
    float xv[2][DM];
    int prev[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long k = min(k0 + 64 * j, hi - 1);
#pragma unroll
      for (int i = 0; i < DM; ++i) xv[j][i] = i < d ? u[k * d + i] : 0.f;
      prev[j] = r > 0 ? side[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long k = k0 + 64 * j;
      if (k >= hi) continue;
      const double da = sqdist_pt<DM>(xv[j], ca, d), db = sqdist_pt<DM>(xv[j], cb, d);
      const int s = da <= db ? 0 : 1;
      if (r > 0 && prev[j] != s) ch = 1;
      side[k] = static_cast<unsigned char>(s);
      n1 += s;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          const double xi = static_cast<double>(xv[j][i]);
          if (s) sb[i] += xi; else sa[i] += xi;
        }
    }
  }
  double* out = w->part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double ta = wave_sum(sa[i]), tb = wave_sum(sb[i]);
      if (lane == 0) { out[i] = ta; out[d + i] = tb; }
    }
  double fn = static_cast<double>(n1), fc = static_cast<double>(ch);
  fn = wave_sum(fn);
  fc = wave_sum(fc);
  if (lane == 0) { out[2 * d] = fn; out[2 * d + 1] = fc; }
}

// after Lloyd pass r: stop when nothing changed (r > 0) or after `iters`
// updates; otherwise the centres become the side means (one more update)
__global__ void __launch_bounds__(256)
k_cl_update(long N, int d, int groups, int r, int iters, double* __restrict__ centres, CLWork* __restrict__ w) {
  __shared__ double red[256 * 33];
  __shared__ int s_stop;
  if (w->st.done) return;
  const int i = threadIdx.x;
  __shared__ double cnt[32], sa[32], sb[32];
  sum_partials(w, groups, 2 * d, 2, red, cnt);   // side-1 count, changed flags
  sum_partials(w, groups, 0, d, red, sa);
  sum_partials(w, groups, d, d, red, sb);
  const double n1 = cnt[0], n0 = static_cast<double>(N) - n1;
  if (i == 0) {
    s_stop = (r > 0 && cnt[1] == 0.0) || r == iters;
    w->st.passes += 1;
    w->st.n1 = static_cast<int>(n1);
    w->st.n0 = static_cast<int>(n0);
  }
  __syncthreads();
  if (!s_stop && i < d) {
    if (n0 > 0.0) w->st.ca[i] = sa[i] / n0;
    if (n1 > 0.0) w->st.cb[i] = sb[i] / n1;
  }
  __syncthreads();
  if (s_stop) {
    if (i < d) { centres[i] = w->st.ca[i]; centres[kMaxD + i] = w->st.cb[i]; }
    if (i == 0) { w->st.done = 1; w->st.iters_used = r; }
  } else if (i == 0) {
    w->st.iters_used = r + 1;
  }
}

__global__ void k_cl_finish(int* __restrict__ passes, CLWork* __restrict__ w) {
  if (threadIdx.x == 0 && passes) *passes = w->st.passes;
}

hipError_t launch_cluster_split(const float* u, long N, int d, int iters, double* mean, double* cov,
                                double* centres, unsigned char* side, void* work, int* passes, hipStream_t s) {
  if (N < 2 || d < 1 || d > kMaxD || iters < 0) return hipErrorInvalidValue;
  CLWork* w = static_cast<CLWork*>(work);
  const int G = static_cast<int>(std::min<long>(kCLGroups, std::max<long>(1, (N + 255) / 256)));
  const int DM = d <= 2 ? 2 : d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32;
#define NS_CL_DM(K, ...)                                                                   \
  switch (DM) {                                                                              \
    case 2: hipLaunchKernelGGL(K<2>, dim3(G), dim3(64), 0, s, __VA_ARGS__); break;           \
    case 4: hipLaunchKernelGGL(K<4>, dim3(G), dim3(64), 0, s, __VA_ARGS__); break;           \
    case 8: hipLaunchKernelGGL(K<8>, dim3(G), dim3(64), 0, s, __VA_ARGS__); break;           \
    case 16: hipLaunchKernelGGL(K<16>, dim3(G), dim3(64), 0, s, __VA_ARGS__); break;         \
    default: hipLaunchKernelGGL(K<32>, dim3(G), dim3(64), 0, s, __VA_ARGS__); break;         \
  }
  NS_CL_DM(k_cl_sum, u, N, d, w)
  hipLaunchKernelGGL(k_cl_mean, dim3(1), dim3(256), 0, s, N, d, G, mean, w);
  // the register triangle for d <= 12 (78 accumulators at most), LDS beyond
  if (d <= 2) hipLaunchKernelGGL(k_cl_cov_reg<2>, dim3(G), dim3(64), 0, s, u, N, d, mean, w);
  else if (d <= 4) hipLaunchKernelGGL(k_cl_cov_reg<4>, dim3(G), dim3(64), 0, s, u, N, d, mean, w);
  else if (d <= 8) hipLaunchKernelGGL(k_cl_cov_reg<8>, dim3(G), dim3(64), 0, s, u, N, d, mean, w);
  else if (d <= 12) hipLaunchKernelGGL(k_cl_cov_reg<12>, dim3(G), dim3(64), 0, s, u, N, d, mean, w);
  else hipLaunchKernelGGL(k_cl_cov, dim3(G), dim3(64), 0, s, u, N, d, mean, w);
  hipLaunchKernelGGL(k_cl_covred, dim3((d * (d + 1) / 2 + 31) / 32), dim3(256), 0, s, N, d, G, cov, w);
  for (int which = 0; which < 2; ++which) {
    NS_CL_DM(k_cl_far, u, N, d, which, mean, w)
    hipLaunchKernelGGL(k_cl_farred, dim3(1), dim3(256), 0, s, u, d, G, which, w);
  }
  for (int r = 0; r <= iters; ++r) {
    NS_CL_DM(k_cl_lloyd, u, N, d, r, side, w)
    hipLaunchKernelGGL(k_cl_update, dim3(1), dim3(256), 0, s, N, d, G, r, iters, centres, w);
  }
  hipLaunchKernelGGL(k_cl_finish, dim3(1), dim3(64), 0, s, passes, w);
#undef NS_CL_DM
  return hipGetLastError();
}

}  // namespace ns
