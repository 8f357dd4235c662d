// ns_sort.hpp -- sorting of FP64 likelihoods by (order key, slot) inside one
// workgroup, shared by the selection kernel and the end-of-step kernel.
#pragma once
#include "ns_device.hpp"

namespace ns {

__device__ __forceinline__ bool key_less(uint64_t ka, int sa, uint64_t kb, int sb) {
  return ka < kb || (ka == kb && sa < sb);
}

// Bitonic network with the keys in registers: thread t holds elements 2t and
// 2t+1 (128 <= P <= 2048, blockDim.x >= P/2).  Partners at distance j = 1
// are in the same thread, partners in the same wave are exchanged with
// shuffles, and only distances of 128 and more go through LDS.  Threads
// beyond P/2 hold padding: their partners are padding as well (j < P keeps
// the bits above P), and P/2 is a multiple of the wave size, so whole waves
// are either in the network or outside it.  keys / slots: LDS of 2 blockDim.x
// entries; on return the first P hold the sorted (key, slot) pairs.
constexpr int kSmallSort = 2048;

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), mask);
  const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), mask);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// key(i) for i < key.n: the order key of entry i (FP64 likelihood bits)
struct LogLKey {
  const double* logL;
  int n;
  __device__ __forceinline__ uint64_t operator()(int i) const { return order_key(logL[i]); }
};

template <typename KeyOf>
__device__ void sort_small(KeyOf key, int P, uint64_t* keys, int* slots) {
  const int t = threadIdx.x;
  const int i0 = 2 * t, i1 = 2 * t + 1;
  // padding: keys above every finite or infinite logL, distinct slots
  uint64_t k0 = i0 < key.n ? key(i0) : ~0ull;
  uint64_t k1 = i1 < key.n ? key(i1) : ~0ull;
  int s0 = i0, s1 = i1;
  for (int k = 2; k <= P; k <<= 1) {
    const bool up = (i0 & k) == 0;
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 1) {
        if (key_less(k1, s1, k0, s0) == up) {
          const uint64_t tk = k0; k0 = k1; k1 = tk;
          const int ts = s0; s0 = s1; s1 = ts;
        }
        continue;
      }
      uint64_t pk0, pk1;
      int ps0, ps1;
      const int tj = j >> 1;
      if (tj < 64) {
        pk0 = shfl_xor_u64(k0, tj); ps0 = __shfl_xor(s0, tj);
        pk1 = shfl_xor_u64(k1, tj); ps1 = __shfl_xor(s1, tj);
      } else {
        __syncthreads();
        keys[i0] = k0; keys[i1] = k1; slots[i0] = s0; slots[i1] = s1;
        __syncthreads();
        pk0 = keys[i0 ^ j]; ps0 = slots[i0 ^ j];
        pk1 = keys[i1 ^ j]; ps1 = slots[i1 ^ j];
      }
      // the lower element of a pair keeps the smaller key when ascending
      const bool lower = (i0 & j) == 0;
      const bool p0 = key_less(pk0, ps0, k0, s0), p1 = key_less(pk1, ps1, k1, s1);
      if (lower == up ? p0 : !p0) { k0 = pk0; s0 = ps0; }
      if (lower == up ? p1 : !p1) { k1 = pk1; s1 = ps1; }
    }
  }
  __syncthreads();
  keys[i0] = k0; keys[i1] = k1; slots[i0] = s0; slots[i1] = s1;
  __syncthreads();
}

__host__ __device__ inline int sort_width(int N) {
  int P = 1;
  while (P < N) P <<= 1;
  return P < 128 ? 128 : P;
}

}  // namespace ns
