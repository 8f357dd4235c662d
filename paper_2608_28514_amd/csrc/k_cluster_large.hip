// k_cluster_large.hip -- one node of the cluster tree (Sec. 2.1) for point
// sets far beyond one workgroup: mean, unbiased covariance and the k-means
// split (k = 2, Lloyd) of N points, as the tree kernels compute them per node.
//
// Every statistic is one streaming pass over the points: workgroups of four
// waves take contiguous chunks and stage 256 points at a time in LDS (16-byte
// loads, the next two tiles in flight while one is used; an odd point stride
// in LDS so that lanes reading consecutive points hit distinct banks).  Lanes
// accumulate in FP64, waves reduce with a fixed butterfly, one partial per
// workgroup is written, and a single workgroup adds the partials in workgroup
// order (deterministic).
// For d <= 16 the mean and covariance come from one pass of moments about the
// first point c: S = sum (x - c), Q = sum (x - c)(x - c)^T (fused
// multiply-adds), mean = c + S / N,
// cov = (Q - S S^T / N) / (N - 1) (the same quantities as the centred
// definition; the shift keeps the terms at the scale of the spread); for
// d > 16 a centred pass follows the mean pass.
// The split starts from the point farthest from the mean and the point
// farthest from that one (lowest index on ties), assigns a point to the first
// centre on a distance tie, and runs Lloyd updates until no assignment
// changes or after `iters` updates; an empty side keeps its centre.  Passes
// after the stop exit at once.
#include <algorithm>
#include <atomic>
#include "ns_device.hpp"
#include "ns_cluster_large.hpp"

namespace ns {

// amdgpu_waves_per_eu(4) on the moments pass: at most 128 VGPRs, four
// workgroups per CU (for d <= 12; wider points keep their registers)
#define NS_CL_OCC __attribute__((amdgpu_waves_per_eu(DM <= 12 ? 4 : 1)))

constexpr int kCLGroups = 1024;     // workgroups of a pass
constexpr int kCLTile = 256;        // points staged per step (one per thread)
constexpr int kCLPart = 528;        // doubles per partial: max(d + d (d + 1) / 2 (d <= 16), d (d + 1) / 2, 2 d + 2)

struct CLState {
  double ca[kMaxD], cb[kMaxD];
  int ia, ib;
  int done, passes, iters_used;
  int n0, n1;
};

constexpr int kCLFan = 32;          // partial rows per workgroup of a reduction kernel
constexpr int kCLFirst = kCLGroups / kCLFan;

struct CLWork {
  CLState st;
  unsigned int tt;                  // finished workgroups of a reduction kernel
  unsigned int bar;                 // arrivals at the grid barriers of the one-launch split
  double pad[7];
  double part[kCLGroups][kCLPart];  // one partial per workgroup
  double gpart[kCLFirst][kCLPart];  // one partial per group
  double pv[kCLGroups], gpv[kCLFirst];
  long pi[kCLGroups], gpi[kCLFirst];
};

size_t cluster_split_work_bytes() { return sizeof(CLWork); }

// v summed over the wave by the butterfly with partners lane ^ 32, ^ 16, ^ 8,
// ^ 4, ^ 2, ^ 1.  After the first two steps a lane's value depends only on
// lane mod 16, and after each later step only on lane mod o, so the last four
// partners are met by rotating each 16-lane row (DPP), which finds the same
// values as the xor partners: the sums are the butterfly's, bit for bit.
__device__ __forceinline__ double wave_sum(double v) {
  v += __shfl_xor(v, 32);
  v += __shfl_xor(v, 16);
  v += dpp_row_ror<8>(v);
  v += dpp_row_ror<4>(v);
  v += dpp_row_ror<2>(v);
  v += dpp_row_ror<1>(v);
  return v;
}

// Ticket of a reduction level: true in the workgroup that finishes it (the
// counter is reset there for the next pass).
__device__ __forceinline__ bool last_in(unsigned int* ctr, int n, int* s_go) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    *s_go = atomicAdd(ctr, 1u) == static_cast<unsigned int>(n - 1);
    if (*s_go) atomicExch(ctr, 0u);
  }
  __syncthreads();
  if (!*s_go) return false;
  __threadfence();
  return true;
}

// Reduction kernels run on ceil(G / 32) workgroups after a pass wrote its G
// partial rows.  red_sum: workgroup b adds rows 32 b .. 32 b + 31 of part in
// order into gpart[b]; the last workgroup to finish adds the gpart rows in
// order into tot (LDS) and returns true.
__device__ bool red_sum(CLWork* w, int G, int nc, double* tot) {
  __shared__ int s_go;
  const int b = blockIdx.x, g0 = kCLFan * b, gsz = min(kCLFan, G - g0), ng = gridDim.x;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double a = 0.0;
    for (int j0 = 0; j0 < gsz; j0 += 16) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = j0 + j < gsz ? w->part[g0 + j0 + j][c] : 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j0 + j < gsz) a = (j0 + j == 0) ? v[j] : a + v[j];
    }
    w->gpart[b][c] = a;
  }
  if (!last_in(&w->tt, ng, &s_go)) return false;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double a = 0.0;
    for (int j0 = 0; j0 < ng; j0 += 16) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = j0 + j < ng ? w->gpart[j0 + j][c] : 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j0 + j < ng) a = (j0 + j == 0) ? v[j] : a + v[j];
    }
    tot[c] = a;
  }
  __syncthreads();
  return true;
}

// the same for the farthest-point partials (pv, pi): largest value, lowest
// index on ties; the result in *bv, *bi of the returning workgroup (thread 0).
// Each level: thread j < 32 loads entry j, thread 0 scans them in order.
__device__ bool red_argmax(CLWork* w, int G, double* bv, long* bi) {
  __shared__ int s_go;
  __shared__ double sv[kCLFan];
  __shared__ long si[kCLFan];
  const int b = blockIdx.x, g0 = kCLFan * b, gsz = min(kCLFan, G - g0), ng = gridDim.x;
  auto scan = [&](int n, double* v, long* ix) {
    *v = -1.0;
    *ix = 0x7fffffffffffffffL;
    for (int j = 0; j < n; ++j)
      if (sv[j] > *v || (sv[j] == *v && si[j] < *ix)) { *v = sv[j]; *ix = si[j]; }
  };
  if (threadIdx.x < gsz) { sv[threadIdx.x] = w->pv[g0 + threadIdx.x]; si[threadIdx.x] = w->pi[g0 + threadIdx.x]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v;
    long ix;
    scan(gsz, &v, &ix);
    w->gpv[b] = v;
    w->gpi[b] = ix;
  }
  if (!last_in(&w->tt, ng, &s_go)) return false;
  if (threadIdx.x < ng) { sv[threadIdx.x] = w->gpv[threadIdx.x]; si[threadIdx.x] = w->gpi[threadIdx.x]; }
  __syncthreads();
  if (threadIdx.x == 0) scan(ng, bv, bi);
  return true;
}

// chunk of workgroup g: points [lo, hi), lo a multiple of 4 (so that tiles
// start on 16-byte boundaries of an aligned array)
__device__ __forceinline__ void chunk_of(long N, long* lo, long* hi) {
  long per = (N + gridDim.x - 1) / gridDim.x;
  per = (per + 3) & ~3L;
  *lo = min(N, static_cast<long>(blockIdx.x) * per);
  *hi = min(N, *lo + per);
}

// LDS floats of a tile: 256 points at stride d | 1, or the 16-byte copy of
// 256 d floats (d odd), whichever is longer
template <int DM>
constexpr int tile_quads() { return (DM + 3) / 4; }   // float4 loads per thread and tile
template <int DM>
constexpr int tile_floats() {
  return tile_quads<DM>() * 4 * kCLTile > kCLTile * (DM + 1) ? tile_quads<DM>() * 4 * kCLTile : kCLTile * (DM + 1);
}

// Loads of one tile: the nf = nt d floats from flat index f0 (a multiple of 4)
// as float4 r[q] = floats 4 (t + 256 q) .. + 3; floats past nf read as 0.
template <int QF>
__device__ __forceinline__ void tile_fetch(const float* __restrict__ u, long f0, int nf, bool al, float4 (&r)[QF]) {
#pragma unroll
  for (int q = 0; q < QF; ++q) {
    const int e = 4 * (static_cast<int>(threadIdx.x) + kCLTile * q);
    const float* p = u + f0 + e;
    if (al && e + 4 <= nf) {
      r[q] = *reinterpret_cast<const float4*>(p);
    } else {
      r[q].x = e < nf ? p[0] : 0.f;
      r[q].y = e + 1 < nf ? p[1] : 0.f;
      r[q].z = e + 2 < nf ? p[2] : 0.f;
      r[q].w = e + 3 < nf ? p[3] : 0.f;
    }
  }
}

// Stores a fetched tile in LDS, point t at xs + t ds with ds = d | 1.  For
// even d flat float e goes to e + e / d, the quotient by a multiply-shift
// (exact for e < 2^13, d <= 32).
template <int QF>
__device__ __forceinline__ void tile_put(float* xs, int nf, int d, const float4 (&r)[QF]) {
  if (d & 1) {
#pragma unroll
    for (int q = 0; q < QF; ++q) {
      const int e = 4 * (static_cast<int>(threadIdx.x) + kCLTile * q);
      if (e < nf) *reinterpret_cast<float4*>(xs + e) = r[q];
    }
  } else {
    const unsigned int mg = ((1u << 20) + d - 1) / d;
#pragma unroll
    for (int q = 0; q < QF; ++q) {
      const int e = 4 * (static_cast<int>(threadIdx.x) + kCLTile * q);
      const float v[4] = {r[q].x, r[q].y, r[q].z, r[q].w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned int el = static_cast<unsigned int>(e + c);
        if (static_cast<int>(el) < nf) xs[el + ((el * mg) >> 20)] = v[c];
      }
    }
  }
}

// The launcher rounds d up to an even DM (d <= 16), so d >= DM - 1 there:
// told to the compiler, every coordinate guard but the last folds away.
template <int DM>
__device__ __forceinline__ void assume_dm(int d) {
  if constexpr (DM <= 16) __builtin_assume(d >= DM - 1 && d <= DM);
}

// Tile layouts in LDS.  PutF: the floats, point t at xs + t (d | 1).
struct PutF {
  float* xs;
  int d;
  template <int QF>
  __device__ __forceinline__ void operator()(int nf, const float4 (&r)[QF]) const { tile_put<QF>(xs, nf, d, r); }
};

// PutShift: the coordinates as doubles minus the shift cs (LDS, d entries),
// point t at xd + t (d | 1)
struct PutShift {
  double* xd;
  const double* cs;
  int d;
  template <int QF>
  __device__ __forceinline__ void operator()(int nf, const float4 (&r)[QF]) const {
    const unsigned int mg = ((1u << 20) + d - 1) / d, pad = (d & 1) ? 0u : 1u;
#pragma unroll
    for (int q = 0; q < QF; ++q) {
      const int e = 4 * (static_cast<int>(threadIdx.x) + kCLTile * q);
      const float v[4] = {r[q].x, r[q].y, r[q].z, r[q].w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned int el = static_cast<unsigned int>(e + c);
        if (static_cast<int>(el) < nf) {
          const unsigned int pt = (el * mg) >> 20;
          xd[el + pt * pad] = static_cast<double>(v[c]) - cs[el - pt * static_cast<unsigned int>(d)];
        }
      }
    }
  }
};

// Streams points [lo, hi) through LDS, 256 at a time: body(k0, nt, pv) runs
// with points k0 .. k0 + nt - 1 stored by put while the next two tiles load.
// pre (may be null): one byte per point fetched with its tile and handed to
// body as pv (thread t: point k0 + t).
template <int QF, class Put, class Body>
__device__ __forceinline__ void stream_tiles(const float* __restrict__ u, int d, long lo, long hi, const Put& put,
                                             const unsigned char* pre, Body&& body) {
  const bool al = (reinterpret_cast<uintptr_t>(u) & 15) == 0;
  const long n = hi - lo;
  const long ntile = (n + kCLTile - 1) / kCLTile;
  auto nf = [&](long k) { return static_cast<int>(min(static_cast<long>(kCLTile), n - k * kCLTile)) * d; };
  auto fetch = [&](long k, float4 (&r)[QF], int& pb) {
    tile_fetch<QF>(u, (lo + k * kCLTile) * d, nf(k), al, r);
    const long i = lo + k * kCLTile + threadIdx.x;
    pb = (pre != nullptr && i < hi) ? static_cast<int>(pre[i]) : 0;
  };
  float4 ra[QF], rb[QF];
  int pa = 0, pb = 0;
  if (ntile > 0) fetch(0, ra, pa);
  if (ntile > 1) fetch(1, rb, pb);
  for (long k = 0; k < ntile; k += 2) {
    __syncthreads();
    put(nf(k), ra);
    const int va = pa;
    __syncthreads();
    if (k + 2 < ntile) fetch(k + 2, ra, pa);
    body(lo + k * kCLTile, nf(k) / d, va);
    if (k + 1 < ntile) {
      __syncthreads();
      put(nf(k + 1), rb);
      const int vb = pb;
      __syncthreads();
      if (k + 3 < ntile) fetch(k + 3, rb, pb);
      body(lo + (k + 1) * kCLTile, nf(k + 1) / d, vb);
    }
  }
}

// The moment list of a point x (coordinates minus the shift, zero past d):
// entries S_0 .. S_{DM-1}, then Q_ij (j <= i) row by row.  Wave W of the
// workgroup owns the entries e with e % 4 == W, in slot e / 4.
template <int DM>
constexpr int stats_slots() { return (DM + DM * (DM + 1) / 2 + 3) / 4; }

template <int DM, int W>
__device__ __forceinline__ void stats_acc(const double (&x)[DM], int d, double (&acc)[stats_slots<DM>()]) {
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i % 4 == W) acc[i / 4] += x[i];
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const int e = DM + i * (i + 1) / 2 + j;
        if (e % 4 == W) acc[e / 4] = __builtin_fma(x[i], x[j], acc[e / 4]);
      }
}

// wave W's entries over the points of a tile (shifted coordinates in LDS):
// lane l takes points l, l + 64, l + 128, l + 192 (in that order)
template <int DM, int W>
__device__ __forceinline__ void stats_tile(const double* xd, int nt, int d, int ds, int lane,
                                           double (&acc)[stats_slots<DM>()]) {
#pragma unroll 1
  for (int t = lane; t < nt; t += 64) {
    double x[DM];
#pragma unroll
    for (int i = 0; i < DM; ++i) x[i] = i < d ? xd[t * ds + i] : 0.0;
    stats_acc<DM, W>(x, d, acc);
  }
}

// partial columns: S_i at i, Q_ij at d + i (i + 1) / 2 + j
template <int DM, int W>
__device__ __forceinline__ void stats_write(const double (&acc)[stats_slots<DM>()], int d, double* row, int lane) {
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i % 4 == W && i < d) {
      const double v = wave_sum(acc[i / 4]);
      if (lane == 0) row[i] = v;
    }
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const int e = DM + i * (i + 1) / 2 + j;
        if (e % 4 == W) {
          const double v = wave_sum(acc[e / 4]);
          if (lane == 0) row[d + i * (i + 1) / 2 + j] = v;
        }
      }
}

// pass (d <= DM <= 16): moments about the first point.  Every wave takes all
// points of a tile (lane l: points l, l + 64, l + 128, l + 192) for its share
// of the entries.
template <int DM>
__global__ void __launch_bounds__(256) NS_CL_OCC
k_cl_stats(const float* __restrict__ u, long N, int d, CLWork* __restrict__ w) {
  constexpr int QF = tile_quads<DM>();
  __shared__ double xd[kCLTile * (DM + 1)];
  __shared__ double cs[DM];
  long lo, hi;
  assume_dm<DM>(d);
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, ds = d | 1;
  if (threadIdx.x < d) cs[threadIdx.x] = static_cast<double>(u[threadIdx.x]);
  __syncthreads();
  double acc[stats_slots<DM>()];
#pragma unroll
  for (int q = 0; q < stats_slots<DM>(); ++q) acc[q] = 0.0;
  stream_tiles<QF>(u, d, lo, hi, PutShift{xd, cs, d}, nullptr, [&](long, int nt, int) {
    switch (wv) {
      case 0: stats_tile<DM, 0>(xd, nt, d, ds, lane, acc); break;
      case 1: stats_tile<DM, 1>(xd, nt, d, ds, lane, acc); break;
      case 2: stats_tile<DM, 2>(xd, nt, d, ds, lane, acc); break;
      default: stats_tile<DM, 3>(xd, nt, d, ds, lane, acc); break;
    }
  });
  double* row = w->part[blockIdx.x];
  switch (wv) {
    case 0: stats_write<DM, 0>(acc, d, row, lane); break;
    case 1: stats_write<DM, 1>(acc, d, row, lane); break;
    case 2: stats_write<DM, 2>(acc, d, row, lane); break;
    default: stats_write<DM, 3>(acc, d, row, lane); break;
  }
}

// reduction of the moment partials; the last workgroup writes the mean and
// the covariance
__global__ void __launch_bounds__(256)
k_cl_red_stats(const float* __restrict__ u, long N, int d, int G, double* __restrict__ mean,
               double* __restrict__ cov, CLWork* __restrict__ w) {
  __shared__ double tot[16 + 16 * 17 / 2];
  const int np = d * (d + 1) / 2;
  if (!red_sum(w, G, d + np, tot)) return;
  const double n = static_cast<double>(N);
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    int ii = 0, jj = q;
    while (jj > ii) { jj -= ii + 1; ++ii; }
    const double v = (tot[d + q] - tot[ii] * tot[jj] / n) / (n - 1.0);
    cov[ii * d + jj] = v;
    cov[jj * d + ii] = v;
  }
  if (threadIdx.x < d) mean[threadIdx.x] = static_cast<double>(u[threadIdx.x]) + tot[threadIdx.x] / n;
  if (threadIdx.x == 0) w->st.passes = 1;
}

// pass (d > 16): coordinate sums; the last workgroup writes the mean
template <int DM>
__global__ void __launch_bounds__(256)
k_cl_sum(const float* __restrict__ u, long N, int d, CLWork* __restrict__ w) {
  constexpr int QF = tile_quads<DM>();
  __shared__ __align__(16) float xs[tile_floats<DM>()];
  __shared__ double red[4][DM];
  long lo, hi;
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, ds = d | 1;
  double s[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) s[i] = 0.0;
  stream_tiles<QF>(u, d, lo, hi, PutF{xs, d}, nullptr, [&](long, int nt, int) {
    const int t = threadIdx.x;
    if (t < nt)
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) s[i] += static_cast<double>(xs[t * ds + i]);
  });
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double v = wave_sum(s[i]);
      if (lane == 0) red[wv][i] = v;
    }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < d) w->part[blockIdx.x][i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

__global__ void __launch_bounds__(256)
k_cl_red_mean(long N, int d, int G, double* __restrict__ mean, CLWork* __restrict__ w) {
  __shared__ double tot[kMaxD];
  if (!red_sum(w, G, d, tot)) return;
  const int i = threadIdx.x;
  if (i < d) mean[i] = tot[i] / static_cast<double>(N);
  if (i == 0) w->st.passes = 1;
}

// pass (d > 16): centred outer products (lower triangle, row by row):
// points staged in LDS, lanes own entries; workgroups of one wave, chunks as
// above
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

__global__ void __launch_bounds__(256)
k_cl_red_cov(long N, int d, int G, double* __restrict__ cov, CLWork* __restrict__ w) {
  __shared__ double tot[kMaxD * (kMaxD + 1) / 2];
  const int np = d * (d + 1) / 2;
  if (!red_sum(w, G, np, tot)) return;
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    int ii = 0, jj = q;
    while (jj > ii) { jj -= ii + 1; ++ii; }
    const double v = tot[q] / static_cast<double>(N - 1);
    cov[ii * d + jj] = v;
    cov[jj * d + ii] = v;
  }
  if (threadIdx.x == 0) w->st.passes += 1;
}

// pass: farthest point from ref (which = 0: the mean, 1: point ia), lowest index on ties
template <int DM>
__global__ void __launch_bounds__(256)
k_cl_far(const float* __restrict__ u, long N, int d, int which, const double* __restrict__ mean,
         CLWork* __restrict__ w) {
  constexpr int QF = tile_quads<DM>();
  __shared__ __align__(16) float xs[tile_floats<DM>()];
  __shared__ double ref[kMaxD];
  __shared__ double sv[4];
  __shared__ long si[4];
  long lo, hi;
  assume_dm<DM>(d);
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, ds = d | 1;
  if (threadIdx.x < d)
    ref[threadIdx.x] = which == 0 ? mean[threadIdx.x]
                                  : static_cast<double>(u[static_cast<long>(w->st.ia) * d + threadIdx.x]);
  __syncthreads();
  double bv = -1.0;
  long bi = 0x7fffffffffffffffL;
  stream_tiles<QF>(u, d, lo, hi, PutF{xs, d}, nullptr, [&](long k0, int nt, int) {
    const int t = threadIdx.x;
    if (t < nt) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          const double q = static_cast<double>(xs[t * ds + i]) - ref[i];
          s += q * q;
        }
      if (s > bv) { bv = s; bi = k0 + t; }
    }
  });
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const long oi = __shfl_xor(bi, o);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) { sv[wv] = bv; si[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q)
      if (sv[q] > bv || (sv[q] == bv && si[q] < bi)) { bv = sv[q]; bi = si[q]; }
    w->pv[blockIdx.x] = bv;
    w->pi[blockIdx.x] = bi;
  }
}

// reduction of the farthest-point partials; the last workgroup makes the
// chosen point a start centre
__global__ void __launch_bounds__(256)
k_cl_red_far(const float* __restrict__ u, int d, int G, int which, CLWork* __restrict__ w) {
  __shared__ long s_i;
  double bv;
  long bi;
  if (!red_argmax(w, G, &bv, &bi)) return;
  if (threadIdx.x == 0) {
    s_i = bi;
    if (which == 0) w->st.ia = static_cast<int>(bi); else w->st.ib = static_cast<int>(bi);
    w->st.passes += 1;
  }
  __syncthreads();
  if (threadIdx.x < d) {
    const double v = static_cast<double>(u[s_i * d + threadIdx.x]);
    if (which == 0) w->st.ca[threadIdx.x] = v; else w->st.cb[threadIdx.x] = v;
  }
}

// Lloyd pass r: assign with the current centres (pass 0: the start pair),
// note changes, and sum the coordinates of each side
template <int DM>
__global__ void __launch_bounds__(256)
k_cl_lloyd(const float* __restrict__ u, long N, int d, int r, unsigned char* side, CLWork* __restrict__ w) {
  constexpr int QF = tile_quads<DM>();
  __shared__ __align__(16) float xs[tile_floats<DM>()];
  __shared__ double ca[kMaxD], cb[kMaxD];
  __shared__ double red[4][2 * DM + 2];
  if (w->st.done) return;
  long lo, hi;
  assume_dm<DM>(d);
  chunk_of(N, &lo, &hi);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, ds = d | 1;
  if (threadIdx.x < d) { ca[threadIdx.x] = w->st.ca[threadIdx.x]; cb[threadIdx.x] = w->st.cb[threadIdx.x]; }
  __syncthreads();
  double sa[DM], sb[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) { sa[i] = 0.0; sb[i] = 0.0; }
  int n1 = 0, ch = 0;
  stream_tiles<QF>(u, d, lo, hi, PutF{xs, d}, r > 0 ? side : nullptr, [&](long k0, int nt, int prev) {
    const int t = threadIdx.x;
    if (t < nt) {
      double x[DM];
#pragma unroll
      for (int i = 0; i < DM; ++i) x[i] = i < d ? static_cast<double>(xs[t * ds + i]) : 0.0;
      double da = 0.0, db = 0.0;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          const double qa = x[i] - ca[i], qb = x[i] - cb[i];
          da += qa * qa;
          db += qb * qb;
        }
      const int sd = da <= db ? 0 : 1;
      if (r > 0 && prev != sd) ch = 1;
      side[k0 + t] = static_cast<unsigned char>(sd);
      n1 += sd;
      // each side's sum takes the coordinate or an exact zero
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          sa[i] += sd ? 0.0 : x[i];
          sb[i] += sd ? x[i] : 0.0;
        }
    }
  });
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double ta = wave_sum(sa[i]), tb = wave_sum(sb[i]);
      if (lane == 0) { red[wv][i] = ta; red[wv][d + i] = tb; }
    }
  const double fn = wave_sum(static_cast<double>(n1)), fc = wave_sum(static_cast<double>(ch));
  if (lane == 0) { red[wv][2 * d] = fn; red[wv][2 * d + 1] = fc; }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < 2 * d + 2) w->part[blockIdx.x][c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// reduction after Lloyd pass r; the last workgroup stops the split when
// nothing changed (r > 0) or after `iters` updates, and otherwise makes the
// side means the centres (one more update)
__global__ void __launch_bounds__(256)
k_cl_red_lloyd(long N, int d, int G, int r, int iters, double* __restrict__ centres, CLWork* __restrict__ w) {
  __shared__ double tot[2 * kMaxD + 2];
  if (w->st.done) return;
  if (!red_sum(w, G, 2 * d + 2, tot)) return;
  const int c = threadIdx.x;
  const double n1v = tot[2 * d], n0v = static_cast<double>(N) - n1v;
  const bool stop = (r > 0 && tot[2 * d + 1] == 0.0) || r == iters;
  if (!stop && c < d) {
    if (n0v > 0.0) w->st.ca[c] = tot[c] / n0v;
    if (n1v > 0.0) w->st.cb[c] = tot[d + c] / n1v;
  }
  if (stop && c < d) { centres[c] = w->st.ca[c]; centres[kMaxD + c] = w->st.cb[c]; }
  if (c == 0) {
    w->st.passes += 1;
    w->st.n1 = static_cast<int>(n1v);
    w->st.n0 = static_cast<int>(n0v);
    w->st.iters_used = stop ? r : r + 1;
    if (stop) w->st.done = 1;
  }
}

// start of a node: the reduction ticket and the stop flag cleared
__global__ void k_cl_init(CLWork* __restrict__ w) {
  const int t = threadIdx.x;
  if (t == 0) {
    w->tt = 0u;
    w->bar = 0u;
    w->st.done = 0;
    w->st.passes = 0;
    w->st.iters_used = 0;
  }
}

__global__ void k_cl_finish(int* __restrict__ passes, CLWork* __restrict__ w) {
  if (threadIdx.x == 0 && passes) *passes = w->st.passes;
}

// ---------------------------------------------------------------- one launch
// A point set of at most kCoopMaxG tiles takes the mean, the two farthest
// points and the Lloyd passes in one cooperative launch: workgroup g keeps
// tile g (256 points, the same tiles and the same thread-per-point sums as the
// streaming passes) in LDS and registers for the whole split, and after each
// phase the workgroups exchange one partial row each through the workspace
// and a grid barrier.  Every workgroup adds the rows in workgroup order, so
// all of them hold the same totals and take the same decisions.  Partial rows
// alternate between two banks from one exchange to the next, so a row is
// never rewritten while another workgroup may still read it.
constexpr int kCoopMaxG = 64;
constexpr long kCoopSpin = 1L << 24;   // default barrier polls before giving up (never reached by a co-resident grid)

// Grid barrier number k (1, 2, ...): the workgroup's writes before it are
// visible to every workgroup after it.  False after `spin` polls without
// every arrival (s_ok cleared, *fault set when given).
// One release (the arrival) and one acquire (after the wait) per workgroup;
// the wait itself polls with relaxed loads.
__device__ __forceinline__ bool coop_barrier(unsigned int* ctr, unsigned int G, unsigned int k, long spin,
                                             int* fault, int* s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < G * k) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin) {
        *s_ok = 0;
        if (fault) atomicOr(fault, 1);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return *s_ok != 0;
}

// The sum of column c over rows r0 .. r0 + G - 1 of the partials, in row
// order, with sixteen loads in flight at a time.
__device__ __forceinline__ double rows_sum(const CLWork* w, int r0, unsigned int G, int c) {
  double a = 0.0;
  for (unsigned int q0 = 0; q0 < G; q0 += 16) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = q0 + q < G ? w->part[r0 + q0 + q][c] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q0 + q < G) a = (q0 + q == 0) ? v[q] : a + v[q];
  }
  return a;
}

// every lane of a 16-lane row ends with the row's sum (DPP rotations)
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_row_ror<8>(v);
  v += dpp_row_ror<4>(v);
  v += dpp_row_ror<2>(v);
  v += dpp_row_ror<1>(v);
  return v;
}

// the largest value, lowest index on ties, over the wave
__device__ __forceinline__ void wave_argmax(double& bv, long& bi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const long oi = __shfl_xor(bi, o);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
}

template <int DM>
__global__ void __launch_bounds__(256)
k_cl_coop(const float* __restrict__ u, long N, int d, int iters, double* __restrict__ mean,
          double* __restrict__ centres, unsigned char* __restrict__ side, double* __restrict__ cstats,
          int* __restrict__ fault, long spin, CLWork* __restrict__ w) {
  constexpr int QF = tile_quads<DM>();
  __shared__ __align__(16) float xs[tile_floats<DM>()];
  __shared__ double red[16][2 * DM + 2];   // one row per 16-lane row of the workgroup
  __shared__ double cen[2][DM];
  __shared__ double tot[2 * DM + 2];
  __shared__ double sv[4];
  __shared__ long si[4];
  __shared__ long s_best;
  __shared__ int s_ok;
  __shared__ unsigned char sside[kCLTile];
  __shared__ double cmu[2][DM];
  const unsigned int G = gridDim.x;
  const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6, ds = d | 1;
  const int row = t >> 4;            // 16-lane row of the workgroup
  const bool head = (t & 15) == 0;
  // a workgroup's sum of column c: the 16 row sums in row order
  auto wg_sum = [&](int c) {
    double a = red[0][c];
    for (int q = 1; q < 16; ++q) a += red[q][c];
    return a;
  };
  const long lo = static_cast<long>(g) * kCLTile, hi = min(N, lo + kCLTile);
  const int nt = static_cast<int>(hi - lo);
  const bool mine = t < nt;
  if (t == 0) s_ok = 1;
  {
    float4 r[QF];
    tile_fetch<QF>(u, lo * d, nt * d, (reinterpret_cast<uintptr_t>(u) & 15) == 0, r);
    tile_put<QF>(xs, nt * d, d, r);
  }
  __syncthreads();
  double x[DM];
#pragma unroll
  for (int i = 0; i < DM; ++i) x[i] = (mine && i < d) ? static_cast<double>(xs[t * ds + i]) : 0.0;
  unsigned int bk = 0;
  // ---- mean (the row sums in workgroup order, then / N)
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const double v = row16_sum(x[i]);
      if (head) red[row][i] = v;
    }
  __syncthreads();
  if (t < d) w->part[g][t] = wg_sum(t);
  if (!coop_barrier(&w->bar, G, ++bk, spin, fault, &s_ok)) return;
  if (t < d) {
    const double m = rows_sum(w, 0, G, t) / static_cast<double>(N);
    cen[0][t] = m;
    if (g == 0) mean[t] = m;
  }
  __syncthreads();
  // ---- the point farthest from the mean, then the one farthest from it
  // (the reference is cen[0] both times: the mean, then point ia)
  for (int which = 0; which < 2; ++which) {
    double bv = -1.0;
    long bi = 0x7fffffffffffffffL;
    if (mine) {
      double s2 = 0.0;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          const double q = x[i] - cen[0][i];
          s2 += q * q;
        }
      bv = s2;
      bi = lo + t;
    }
    wave_argmax(bv, bi);
    if (lane == 0) { sv[wv] = bv; si[wv] = bi; }
    __syncthreads();
    if (t == 0) {
      for (int q = 1; q < 4; ++q)
        if (sv[q] > bv || (sv[q] == bv && si[q] < bi)) { bv = sv[q]; bi = si[q]; }
      w->pv[which * G + g] = bv;
      w->pi[which * G + g] = bi;
    }
    if (!coop_barrier(&w->bar, G, ++bk, spin, fault, &s_ok)) return;
    if (t < 64) {
      // lane q reads the partial of workgroup q (and q + 64 ...), then the
      // wave takes the largest value, lowest index on ties
      double v = -1.0;
      long ix = 0x7fffffffffffffffL;
      for (unsigned int q = t; q < G; q += 64) {
        const double pv = w->pv[which * G + q];
        const long pi = w->pi[which * G + q];
        if (pv > v || (pv == v && pi < ix)) { v = pv; ix = pi; }
      }
      wave_argmax(v, ix);
      if (t == 0) {
        s_best = ix;
        if (g == 0) { if (which == 0) w->st.ia = static_cast<int>(ix); else w->st.ib = static_cast<int>(ix); }
      }
    }
    __syncthreads();
    // the start centres: ca = point ia (replacing the mean), cb = point ib
    if (t < d) cen[which][t] = static_cast<double>(u[s_best * d + t]);
    __syncthreads();
  }
  // ---- Lloyd: assign with the current centres (a tie to the first), sum the
  // sides; stop at a fixed point or after `iters` updates
  int prev = 0, used = 0;
  double n0f = 0.0, n1f = 0.0;
  for (int r = 0; r <= iters; ++r) {
    int sd = 0, ch = 0;
    if (mine) {
      double da = 0.0, db = 0.0;
#pragma unroll
      for (int i = 0; i < DM; ++i)
        if (i < d) {
          const double qa = x[i] - cen[0][i], qb = x[i] - cen[1][i];
          da += qa * qa;
          db += qb * qb;
        }
      sd = da <= db ? 0 : 1;
      if (r > 0 && prev != sd) ch = 1;
      prev = sd;
    }
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i < d) {
        const double ta = row16_sum(sd ? 0.0 : x[i]), tb = row16_sum(sd ? x[i] : 0.0);
        if (head) { red[row][i] = ta; red[row][d + i] = tb; }
      }
    const double fn = row16_sum(static_cast<double>(sd)), fc = row16_sum(static_cast<double>(ch));
    if (head) { red[row][2 * d] = fn; red[row][2 * d + 1] = fc; }
    __syncthreads();
    const int bank = (r & 1) * static_cast<int>(G);
    if (t < 2 * d + 2) w->part[bank + g][t] = wg_sum(t);
    if (!coop_barrier(&w->bar, G, ++bk, spin, fault, &s_ok)) return;
    if (t < 2 * d + 2) tot[t] = rows_sum(w, bank, G, t);
    __syncthreads();
    const double n1v = tot[2 * d], n0v = static_cast<double>(N) - n1v;
    const bool stop = (r > 0 && tot[2 * d + 1] == 0.0) || r == iters;
    used = stop ? r : r + 1;
    n0f = n0v;
    n1f = n1v;
    if (!stop && t < d) {
      if (n0v > 0.0) cen[0][t] = tot[t] / n0v;
      if (n1v > 0.0) cen[1][t] = tot[d + t] / n1v;
    }
    __syncthreads();
    if (stop) {
      if (g == 0 && t == 0) {
        w->st.n1 = static_cast<int>(n1v);
        w->st.n0 = static_cast<int>(n0v);
        w->st.iters_used = used;
        w->st.done = 1;
      }
      break;
    }
  }
  if (mine) side[lo + t] = static_cast<unsigned char>(prev);
  if (g == 0 && t < d) {
    centres[t] = cen[0][t];
    centres[kMaxD + t] = cen[1][t];
  }
  if (cstats == nullptr) return;
  // ---- the two children (the leaves of a depth-1 tree): count, mean (the
  // side sums of the final assignment / count) and unbiased covariance about
  // that mean.  Thread-per-pair sums over the workgroup's points, one partial
  // row per child and workgroup, added in workgroup order by workgroup 0.
  if (mine) sside[t] = static_cast<unsigned char>(prev);
  if (t < d) {
    cmu[0][t] = n0f > 0.0 ? tot[t] / n0f : 0.0;
    cmu[1][t] = n1f > 0.0 ? tot[d + t] / n1f : 0.0;
  }
  __syncthreads();
  const int np = d * (d + 1) / 2;
  for (int p = t; p < 2 * np; p += 256) {
    const int c = p >= np ? 1 : 0;
    const int pc = p - c * np;
    int i = 0, j = pc;
    while (j > i) { j -= i + 1; ++i; }
    double acc = 0.0;
    for (int k = 0; k < nt; ++k)
      if (sside[k] == c) {
        const double a = static_cast<double>(xs[k * ds + i]) - cmu[c][i];
        const double b = static_cast<double>(xs[k * ds + j]) - cmu[c][j];
        acc += a * b;
      }
    w->part[(2 + c) * static_cast<int>(G) + g][pc] = acc;
  }
  if (!coop_barrier(&w->bar, G, ++bk, spin, fault, &s_ok)) return;
  if (g != 0) return;
  // cstats: counts [0..2), means [2 + 32 c ..), covariances [66 + 1024 c ..) (stride d)
  if (t < 2) cstats[t] = t == 0 ? n0f : n1f;
  if (t < d) {
    cstats[2 + t] = cmu[0][t];
    cstats[2 + 32 + t] = cmu[1][t];
  }
  for (int p = t; p < 2 * np; p += 256) {
    const int c = p >= np ? 1 : 0;
    const int pc = p - c * np;
    int i = 0, j = pc;
    while (j > i) { j -= i + 1; ++i; }
    const double nc = c == 0 ? n0f : n1f;
    const double v = nc >= 2.0 ? rows_sum(w, (2 + c) * static_cast<int>(G), G, pc) / (nc - 1.0) : 0.0;
    double* C = cstats + 66 + 1024 * c;
    C[i * d + j] = v;
    C[j * d + i] = v;
  }
}

// Workgroups of 256 threads of kernel k resident at once on the current
// device (CUs times the occupancy), cached per device and width; 0 if the
// runtime cannot tell.
template <int DM>
static int lloyd_resident() {
  static std::atomic<int> cache[16];   // zero-initialised (static storage)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0, nb = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_cl_lloyd<DM>), 256, 0) !=
            hipSuccess)
      return 0;
    v = cus * nb;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

// Co-resident workgroups of k_cl_coop<DM> on the current device (cached).
template <int DM>
static int coop_resident() {
  static std::atomic<int> cache[16];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0, nb = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_cl_coop<DM>), 256, 0) !=
            hipSuccess)
      return 0;
    v = cus * nb;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

hipError_t launch_cluster_split_coop(const float* u, long N, int d, int iters, double* mean, double* cov,
                                     double* centres, unsigned char* side, double* cstats, void* work,
                                     int* fault, int wait_limit, hipStream_t s) {
  const long G = (N + kCLTile - 1) / kCLTile;
  if (N < 2 || d <= 16 || d > kMaxD || iters < 0 || G > kCoopMaxG) return hipErrorNotSupported;
  const int DM = d <= 24 ? 24 : 32;
  if ((DM == 24 ? coop_resident<24>() : coop_resident<32>()) < G) return hipErrorNotSupported;
  CLWork* w = static_cast<CLWork*>(work);
  hipLaunchKernelGGL(k_cl_init, dim3(1), dim3(64), 0, s, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  long spin = wait_limit > 0 ? wait_limit : kCoopSpin;
  void* args[] = {const_cast<float**>(&u), &N, &d, &iters, &mean, &centres, &side, &cstats, &fault, &spin, &w};
  e = hipLaunchCooperativeKernel(DM == 24 ? reinterpret_cast<const void*>(k_cl_coop<24>)
                                          : reinterpret_cast<const void*>(k_cl_coop<32>),
                                 dim3(static_cast<unsigned>(G)), dim3(256), args, 0, s);
  if (e != hipSuccess) return e;
  // the covariance about that mean: the streaming pass, a workgroup per 64 points
  const int Gc = static_cast<int>(std::min<long>(kCLGroups, std::max<long>(1, (N + 63) / 64)));
  hipLaunchKernelGGL(k_cl_cov, dim3(Gc), dim3(64), 0, s, u, N, d, mean, w);
  hipLaunchKernelGGL(k_cl_red_cov, dim3((Gc + kCLFan - 1) / kCLFan), dim3(256), 0, s, N, d, Gc, cov, w);
  return hipGetLastError();
}

hipError_t launch_cluster_split(const float* u, long N, int d, int iters, double* mean, double* cov,
                                double* centres, unsigned char* side, void* work, int* passes, hipStream_t s) {
  if (N < 2 || d < 1 || d > kMaxD || iters < 0) return hipErrorInvalidValue;
  CLWork* w = static_cast<CLWork*>(work);
  const int G = static_cast<int>(std::min<long>(kCLGroups, std::max<long>(1, (N + kCLTile - 1) / kCLTile)));
  // the dimension rounded up to even (24 and 32 beyond 16): register arrays of that length
  const int DM = d <= 16 ? (d + 1) & ~1 : d <= 24 ? 24 : 32;
#define NS_CL_CASE(K, M, ...) \
  case M: hipLaunchKernelGGL(K<M>, dim3(G), dim3(256), 0, s, __VA_ARGS__); break;
#define NS_CL_CASE_G(K, GG, M, ...) \
  case M: hipLaunchKernelGGL(K<M>, dim3(GG), dim3(256), 0, s, __VA_ARGS__); break;
#define NS_CL_DM(K, ...)                                                                           \
  switch (DM) {                                                                                      \
    NS_CL_CASE(K, 2, __VA_ARGS__) NS_CL_CASE(K, 4, __VA_ARGS__) NS_CL_CASE(K, 6, __VA_ARGS__)       \
    NS_CL_CASE(K, 8, __VA_ARGS__) NS_CL_CASE(K, 10, __VA_ARGS__) NS_CL_CASE(K, 12, __VA_ARGS__)     \
    NS_CL_CASE(K, 14, __VA_ARGS__) NS_CL_CASE(K, 16, __VA_ARGS__) NS_CL_CASE(K, 24, __VA_ARGS__)    \
    default: hipLaunchKernelGGL(K<32>, dim3(G), dim3(256), 0, s, __VA_ARGS__); break;                \
  }
#define NS_CL_DM16(K, ...)                                                                         \
  switch (DM) {                                                                                      \
    NS_CL_CASE(K, 2, __VA_ARGS__) NS_CL_CASE(K, 4, __VA_ARGS__) NS_CL_CASE(K, 6, __VA_ARGS__)       \
    NS_CL_CASE(K, 8, __VA_ARGS__) NS_CL_CASE(K, 10, __VA_ARGS__) NS_CL_CASE(K, 12, __VA_ARGS__)     \
    NS_CL_CASE(K, 14, __VA_ARGS__) default: hipLaunchKernelGGL(K<16>, dim3(G), dim3(256), 0, s, __VA_ARGS__); break; \
  }
  const int R = (G + kCLFan - 1) / kCLFan;   // reduction workgroups
  hipLaunchKernelGGL(k_cl_init, dim3(1), dim3(64), 0, s, w);
  if (d <= 16) {
    NS_CL_DM16(k_cl_stats, u, N, d, w)
    hipLaunchKernelGGL(k_cl_red_stats, dim3(R), dim3(256), 0, s, u, N, d, G, mean, cov, w);
  } else {
    hipLaunchKernelGGL(k_cl_sum<32>, dim3(G), dim3(256), 0, s, u, N, d, w);
    hipLaunchKernelGGL(k_cl_red_mean, dim3(R), dim3(256), 0, s, N, d, G, mean, w);
    // one wave per workgroup: a workgroup per 64 points (up to kCLGroups), so
    // that small point sets still spread over many CUs
    const int Gc = static_cast<int>(std::min<long>(kCLGroups, std::max<long>(1, (N + 63) / 64)));
    hipLaunchKernelGGL(k_cl_cov, dim3(Gc), dim3(64), 0, s, u, N, d, mean, w);
    hipLaunchKernelGGL(k_cl_red_cov, dim3((Gc + kCLFan - 1) / kCLFan), dim3(256), 0, s, N, d, Gc, cov, w);
  }
  for (int which = 0; which < 2; ++which) {
    NS_CL_DM(k_cl_far, u, N, d, which, mean, w)
    hipLaunchKernelGGL(k_cl_red_far, dim3(R), dim3(256), 0, s, u, d, G, which, w);
  }
  // the Lloyd passes hold more registers: their grid is what the device keeps
  // resident at once (one round of workgroups, no tail)
  int res = 0;
  switch (DM) {
    case 2: res = lloyd_resident<2>(); break;
    case 4: res = lloyd_resident<4>(); break;
    case 6: res = lloyd_resident<6>(); break;
    case 8: res = lloyd_resident<8>(); break;
    case 10: res = lloyd_resident<10>(); break;
    case 12: res = lloyd_resident<12>(); break;
    case 14: res = lloyd_resident<14>(); break;
    case 16: res = lloyd_resident<16>(); break;
    case 24: res = lloyd_resident<24>(); break;
    default: res = lloyd_resident<32>(); break;
  }
  const int GL = res > 0 ? std::min(G, res) : G, RL = (GL + kCLFan - 1) / kCLFan;
  for (int r = 0; r <= iters; ++r) {
    switch (DM) {
      NS_CL_CASE_G(k_cl_lloyd, GL, 2, u, N, d, r, side, w) NS_CL_CASE_G(k_cl_lloyd, GL, 4, u, N, d, r, side, w)
      NS_CL_CASE_G(k_cl_lloyd, GL, 6, u, N, d, r, side, w) NS_CL_CASE_G(k_cl_lloyd, GL, 8, u, N, d, r, side, w)
      NS_CL_CASE_G(k_cl_lloyd, GL, 10, u, N, d, r, side, w) NS_CL_CASE_G(k_cl_lloyd, GL, 12, u, N, d, r, side, w)
      NS_CL_CASE_G(k_cl_lloyd, GL, 14, u, N, d, r, side, w) NS_CL_CASE_G(k_cl_lloyd, GL, 16, u, N, d, r, side, w)
      NS_CL_CASE_G(k_cl_lloyd, GL, 24, u, N, d, r, side, w)
      default: hipLaunchKernelGGL(k_cl_lloyd<32>, dim3(GL), dim3(256), 0, s, u, N, d, r, side, w); break;
    }
    hipLaunchKernelGGL(k_cl_red_lloyd, dim3(RL), dim3(256), 0, s, N, d, GL, r, iters, centres, w);
  }
  hipLaunchKernelGGL(k_cl_finish, dim3(1), dim3(64), 0, s, passes, w);
#undef NS_CL_DM
#undef NS_CL_DM16
#undef NS_CL_CASE
#undef NS_CL_CASE_G
  return hipGetLastError();
}

}  // namespace ns
