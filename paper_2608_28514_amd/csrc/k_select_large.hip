// k_select_large.hip -- the m worst of N likelihoods for N far beyond one
// workgroup (Algorithm 1's selection, "sorted", at scale).
//
// Radix select on the composite (order key, index): the FP64 order key is
// resolved from its top bits in 12-bit digits (then 4), and when the key alone
// cannot separate the m-th entry (ties) the index follows in 12-bit digits.
// Every digit costs one streaming pass over logL: each workgroup builds a
// histogram of the digit among the entries that share the resolved prefix (in
// LDS) and writes it out; a small kernel sums the partial histograms, and
// every workgroup of the next launch picks from the totals the bin that holds
// the m-th entry (the same pick in each, so no workgroup waits on another and
// no kernel needs a device-wide fence).  Once at most kSelCap entries lie at
// or below the resolved prefix, one more pass collects them, and each
// candidate's rank among them by (key, index) places the first m indices.
// The result equals a stable sort of (canon(logL), index).
#include <algorithm>
#include <mutex>
#include "ns_device.hpp"
#include "ns_select_large.hpp"

namespace ns {

constexpr int kRBits = 12, kRBins = 1 << kRBits;
constexpr int kSelCap = 8192;      // candidates sorted by the last kernel
constexpr int kSelMaxM = 4096;
constexpr int kSelLevels = 9;      // key digits 52, 40, 28, 16, 4, 0; index digits 20, 8, 0
constexpr int kSelGroups = 512;    // workgroups of a histogram pass (one partial histogram each)

struct SelState {
  unsigned long long kprefix;  // resolved key bits (those at and above kshift)
  unsigned int sprefix;        // resolved index bits (at and above sshift)
  int kshift;                  // 64: no key bit resolved yet
  int sshift;                  // 32: no index bit resolved yet
  int below;                   // entries strictly below the resolved prefix
  int done;                    // at most kSelCap entries at or below the prefix
  int passes;                  // streaming passes over logL so far
};

struct SelWork {
  // slot[l]: the state before digit l (slot[0] from the init kernel, slot[l]
  // written by workgroup 0 of digit l's histogram launch); slot[kSelLevels]:
  // the final state, written by the collect pass
  SelState slot[kSelLevels + 1];
  int ncand;                   // entries collected
  unsigned int pad[31];
  alignas(16) unsigned int hist[kRBins];   // totals of the last summed digit
  alignas(16) unsigned int part[kSelGroups][kRBins];
  unsigned long long ckey[kSelCap];
  int cidx[kSelCap];
};

__host__ __device__ constexpr size_t sel_work_bytes() { return sizeof(SelWork); }

struct Level {
  int slot_phase, shift, width;
};
__host__ __device__ inline Level sel_level(int l) {
  const Level L[kSelLevels] = {{0, 52, 12}, {0, 40, 12}, {0, 28, 12}, {0, 16, 12}, {0, 4, 12}, {0, 0, 4},
                               {1, 20, 12}, {1, 8, 12}, {1, 0, 8}};
  return L[l];
}

// entry relative to the resolved prefix: -1 below, 0 in it, 1 above
__device__ __forceinline__ int sel_rel(unsigned long long key, unsigned int idx, const SelState& s) {
  if (s.kshift == 64) return 0;
  const unsigned long long kh = key >> s.kshift;
  if (kh != s.kprefix) return kh < s.kprefix ? -1 : 1;
  if (s.sshift == 32) return 0;
  const unsigned int ih = idx >> s.sshift;
  if (ih != s.sprefix) return ih < s.sprefix ? -1 : 1;
  return 0;
}

__global__ void k_rsel_init(long N, int m, SelWork* w) {
  for (int b = threadIdx.x; b < kRBins; b += blockDim.x) w->hist[b] = 0u;
  if (threadIdx.x == 0) {
    SelState s{};
    s.kprefix = 0ull;
    s.sprefix = 0u;
    s.kshift = 64;
    s.sshift = 32;
    s.below = 0;
    s.done = N <= kSelCap ? 1 : 0;
    s.passes = 0;
    w->slot[0] = s;
    w->ncand = 0;
  }
}

// The pick of digit `level` from its totals (w->hist), by every thread of a
// workgroup (NB consecutive bins per thread, NB * blockDim.x == kRBins): an
// inclusive scan (thread totals within each wave, then the wave totals)
// finds the first bin where below + cum >= m; each thread returns the
// advanced state.
template <int NB>
__device__ SelState pick_digit(const SelState& s, int level, int m, const SelWork* __restrict__ w) {
  __shared__ unsigned int wsum[16];
  __shared__ int s_bin, s_before;
  __shared__ unsigned int s_cnt;
  const int tt = threadIdx.x, ln = tt & 63, wq = tt >> 6;
  unsigned int hb[NB];
#pragma unroll
  for (int r = 0; r < NB / 4; ++r) {
    const uint4 hv = reinterpret_cast<const uint4*>(w->hist)[NB / 4 * tt + r];
    hb[4 * r] = hv.x;
    hb[4 * r + 1] = hv.y;
    hb[4 * r + 2] = hv.z;
    hb[4 * r + 3] = hv.w;
  }
  unsigned int run = 0u;
#pragma unroll
  for (int q = 0; q < NB; ++q) run += hb[q];
  unsigned int inc = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned int y = __shfl_up(inc, o);
    if (ln >= o) inc += y;
  }
  if (ln == 63) wsum[wq] = inc;
  __syncthreads();
  unsigned int before = inc - run;
  for (int q = 0; q < wq; ++q) before += wsum[q];
  const long need = static_cast<long>(m) - s.below;
  unsigned int c = before;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (static_cast<long>(c) < need && static_cast<long>(c + hb[q]) >= need) {
      s_bin = NB * tt + q;
      s_before = static_cast<int>(c);
      s_cnt = hb[q];
    }
    c += hb[q];
  }
  __syncthreads();
  const Level L = sel_level(level);
  const int bin = s_bin;
  SelState n = s;
  if (L.slot_phase) {
    n.sprefix = (n.sshift == 32) ? static_cast<unsigned int>(bin) : ((n.sprefix << L.width) | bin);
    n.sshift = L.shift;
  } else {
    n.kprefix = (n.kshift == 64) ? static_cast<unsigned long long>(bin)
                                 : ((n.kprefix << L.width) | static_cast<unsigned long long>(bin));
    n.kshift = L.shift;
  }
  n.below = s.below + s_before;
  n.done = (static_cast<long>(n.below) + s_cnt <= kSelCap) ? 1 : 0;
  n.passes = s.passes + 1;
  __syncthreads();   // the LDS words above are reused by the next call
  return n;
}

// One digit, pass 1 of 2: each workgroup counts the digit of the entries in
// the resolved prefix and writes its partial histogram.  Each thread loads
// eight pairs of likelihoods (16-byte loads) before counting them.  The LDS
// histogram is kept in four interleaved copies (bin b, copy c at 4 b + c, so
// the copies of a bin sit in four banks), lane l adding to copy l & 3: lanes
// of a wave that share a digit (likelihoods often share their leading bits)
// then meet at most 16 to an address; the copies are summed at the end.
// Workgroups of 1024 threads (16 waves).
__global__ void __launch_bounds__(1024)
k_rsel_hist(const double* __restrict__ logL, long N, int m, int level, SelWork* __restrict__ w) {
  __shared__ uint4 lh4[kRBins];
  unsigned int* lh = reinterpret_cast<unsigned int*>(lh4);
  // the state before this digit: the previous digit's pick, made here
  SelState s = w->slot[level > 0 ? level - 1 : 0];
  if (level > 0) {
    if (!s.done) s = pick_digit<kRBins / 1024>(s, level - 1, m, w);
    if (blockIdx.x == 0 && threadIdx.x == 0) w->slot[level] = s;
  }
  if (s.done) return;
  const Level L = sel_level(level);
  const unsigned int mask = (1u << L.width) - 1u;
  const unsigned int cp = threadIdx.x & 3;
  for (int b = threadIdx.x; b < kRBins; b += blockDim.x) lh4[b] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const long npair = (N + 1) >> 1;
  const long stride = static_cast<long>(gridDim.x) * blockDim.x;
  const double2* lp = reinterpret_cast<const double2*>(logL);
  for (long p0 = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; p0 < npair; p0 += 8 * stride) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long p = min(p0 + q * stride, npair - 1);
      if (2 * p + 1 < N) {
        v[q] = lp[p];
      } else {
        v[q].x = logL[2 * p];
        v[q].y = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const long i = 2 * (p0 + q * stride) + h;
        if (p0 + q * stride < npair && i < N) {
          const unsigned long long key = order_key(h ? v[q].y : v[q].x);
          if (sel_rel(key, static_cast<unsigned int>(i), s) == 0) {
            const unsigned int dg = L.slot_phase ? ((static_cast<unsigned int>(i) >> L.shift) & mask)
                                                 : static_cast<unsigned int>((key >> L.shift) & mask);
            atomicAdd(&lh[4 * dg + cp], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  unsigned int* out = w->part[blockIdx.x];
  for (int b = threadIdx.x; b < kRBins; b += blockDim.x) {
    const uint4 c = lh4[b];
    out[b] = ((c.x + c.y) + c.z) + c.w;
  }
}

// One digit, pass 2 of 2: the partial histograms summed per bin into the
// totals the next launch picks from.
__global__ void __launch_bounds__(256)
k_rsel_reduce(int groups, int level, SelWork* __restrict__ w) {
  __shared__ unsigned int qs[256];
  if (w->slot[level].done) return;
  // 64 bins per workgroup (gridDim.x * 64 == kRBins); the four waves take
  // every fourth partial (32 loads in flight), then their four sums are added
  // in wave order.
  const int b = blockIdx.x * 64 + (threadIdx.x & 63), qq = threadIdx.x >> 6;
  unsigned int t = 0u;
  for (int g0 = qq; g0 < groups; g0 += 4 * 32) {
    unsigned int v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = w->part[min(g0 + 4 * j, groups - 1)][b];
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if (g0 + 4 * j < groups) t += v[j];
  }
  qs[threadIdx.x] = t;
  __syncthreads();
  if (qq == 0) w->hist[b] = ((qs[threadIdx.x] + qs[64 + threadIdx.x]) + qs[128 + threadIdx.x]) + qs[192 + threadIdx.x];
}

// Every entry at or below the resolved prefix (at most kSelCap) into the
// candidate list, one atomic per wave.
__global__ void __launch_bounds__(256)
k_rsel_collect(const double* __restrict__ logL, long N, int m, SelWork* __restrict__ w) {
  // the last digit's pick, if the digits ran out before the count fell to kSelCap
  SelState s = w->slot[kSelLevels - 1];
  if (!s.done) s = pick_digit<kRBins / 256>(s, kSelLevels - 1, m, w);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SelState f = s;
    f.passes = s.passes + 1;   // this pass
    w->slot[kSelLevels] = f;
  }
  const long stride = static_cast<long>(gridDim.x) * blockDim.x;
  const int lane = threadIdx.x & 63;
  const long n_up = (N + 63) / 64 * 64;   // whole waves run every iteration (ballots)
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_up; i += stride) {
    unsigned long long key = 0ull;
    bool take = false;
    if (i < N) {
      key = order_key(logL[i]);
      take = sel_rel(key, static_cast<unsigned int>(i), s) <= 0;
    }
    const unsigned long long bal = __ballot(take);
    if (!bal) continue;
    int base = 0;
    if (lane == 0) base = atomicAdd(&w->ncand, __popcll(bal));
    base = __shfl(base, 0);
    if (take) {
      const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
      if (pos < kSelCap) {
        w->ckey[pos] = key;
        w->cidx[pos] = static_cast<int>(i);
      }
    }
  }
}

// The candidates ranked by (key, index): one wave per candidate (grid-stride
// over the candidates) counts the candidates before it, eight loads per lane
// in flight; a candidate of rank r < m writes its index to out[r].  Keys
// with their indices are distinct, so the ranks are 0 .. n - 1.
__global__ void __launch_bounds__(256)
k_rsel_rank(int m, const SelWork* __restrict__ w, int* __restrict__ out, int* __restrict__ passes) {
  const int n = min(w->ncand, kSelCap);
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), nwaves = gridDim.x * (blockDim.x >> 6);
  for (int c = wave; c < n; c += nwaves) {
    const unsigned long long kc = w->ckey[c];
    const int ic = w->cidx[c];
    int before = 0;
    for (int j0 = 0; j0 < n; j0 += 8 * 64) {
      unsigned long long kj[8];
      int ij[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = min(j0 + 64 * q + lane, n - 1);
        kj[q] = w->ckey[j];
        ij[q] = w->cidx[j];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool lt = j0 + 64 * q + lane < n && (kj[q] < kc || (kj[q] == kc && ij[q] < ic));
        before += __popcll(__ballot(lt));
      }
    }
    if (lane == 0 && before < m) out[before] = ic;
  }
  if (passes && blockIdx.x == 0 && threadIdx.x == 0) *passes = w->slot[kSelLevels].passes;
}

size_t select_large_work_bytes() { return sel_work_bytes(); }

// Workspace of the allocation-free selection: one SelWork per device, held
// until the process ends.  In host code `scratch` only names the symbol: its
// device address, different on every device, comes from hipGetSymbolAddress
// (made once per device, with that device current) and is the only handle
// host code passes on.  Every call on a device shares this memory, so calls
// that overlap in time on one device race; k_rsel_init clears what the
// passes read before they write it.
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[sizeof(SelWork)];

hipError_t select_large_static_work(void** out) {
  static std::mutex mu;
  static void* ptr[kScratchDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t launch_select_large(const double* logL, long N, int m, int* out, void* work, int* passes,
                               hipStream_t s) {
  if (m < 1 || m > kSelMaxM || m > N) return hipErrorInvalidValue;
  SelWork* w = static_cast<SelWork*>(work);
  hipLaunchKernelGGL(k_rsel_init, dim3(1), dim3(256), 0, s, N, m, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long npair = (N + 1) / 2;
  const int grid = static_cast<int>(std::min<long>(kSelGroups, std::max<long>(1, (npair + 2047) / 2048)));
  for (int l = 0; l < kSelLevels; ++l) {
    hipLaunchKernelGGL(k_rsel_hist, dim3(grid), dim3(1024), 0, s, logL, N, m, l, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rsel_reduce, dim3(kRBins / 64), dim3(256), 0, s, grid, l, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int cgrid = static_cast<int>(std::min<long>(2048, std::max<long>(1, (N + 255) / 256)));
  hipLaunchKernelGGL(k_rsel_collect, dim3(cgrid), dim3(256), 0, s, logL, N, m, w);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rsel_rank, dim3(256), dim3(256), 0, s, m, w, out, passes);
  return hipGetLastError();
}

}  // namespace ns
