// k_gemm.hip -- dense layers of the emulator and surrogate networks.
//
// C[M x N] = epilogue( sum_k A(r, k) B(k, n) ), with strided operands
//   A(r, k) = A[r*sar + k*sak]   (FP32)
//   B(k, n) = B[n*sbn + k*sbk]   (FP32)
// so that the forward pass (A row major, B = W^T), dW = H^T dZ and
// dH = dZ W^T all use the same kernel.  Epilogue: + bias[n], optional tanh /
// SiLU, optional store of the pre-activation Z.
//
// Modes:
//  * kF32   -- FP32 FMA on the vector ALU (4x4 register blocking).
//  * kBF16S -- MFMA v_mfma_f32_16x16x32_bf16 with FP32 accumulation; every A
//              value is split into three bfloat16 terms (hi + mid + lo, which
//              carries ~24 significant bits) and B is rounded once to
//              bfloat16, so for bfloat16-valued weights the product matches an
//              FP32 GEMM up to the accumulation order.
//  * kBF16  -- MFMA with A and B each rounded once to bfloat16.
// Tiles: 64 x 64 outputs per 256-thread workgroup, K in steps of 32 staged
// through LDS; each wave owns a 32 x 32 quadrant (2 x 2 MFMA tiles).
#include "ns_internal.hpp"
#include "ns_gemm.hpp"

namespace ns {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

// rows per call from which the hidden and output layers use 32 x 64 blocks
// per wave; workgroup tiles (64 x 128 for hidden layers, 128 x 128 for the
// output layer) once a layer has this many of them (one per CU)
constexpr int kFragWideRows = 4096;
constexpr int kFragTileMin = 256;

// Workgroups are dealt to the eight XCDs round-robin (workgroup b on XCD
// b % 8), each XCD with its own L2.  The block a workgroup computes is taken
// from a renumbering that gives every XCD a contiguous range of blocks, so the
// column blocks of one row block (which share its activation fragments) run
// on the same XCD; the last G % 8 workgroups keep their own number.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3;
  return b < 8 * q ? (b & 7) * q + (b >> 3) : b;
}

constexpr int kTM = 64, kTN = 64, kTK = 32;
constexpr int kLdsK = kTK + 4;  // padded row stride (floats)

__device__ __forceinline__ float act_fwd(int act, float z) {
  if (act == kActTanh) return tanhf(z);
  if (act == kActSilu) return z / (1.0f + expf(-z));
  return z;
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }
__device__ __forceinline__ float from_bf16(__bf16 x) { return static_cast<float>(x); }

// x = hi + mid + lo, each a bfloat16 (three planes of `plane` elements each).
__device__ __forceinline__ void store_split(__bf16* out, long plane, long idx, float x) {
  const __bf16 h = to_bf16(x);
  const float r1 = x - from_bf16(h);
  const __bf16 m = to_bf16(r1);
  out[idx] = h;
  out[plane + idx] = m;
  out[2 * plane + idx] = to_bf16(r1 - from_bf16(m));
}

template <int MODE>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const float* __restrict__ A, long sar, long sak,
       const float* __restrict__ B, long sbn, long sbk, const float* __restrict__ bias, int act,
       float* __restrict__ C, long ldc, float* __restrict__ Z, long ldz, const int* __restrict__ gate,
       const int* __restrict__ dM, __bf16* __restrict__ Csplit, long plane, int kchunk) {
  if (gate && *gate == 0) return;
  if (dM) M = min(M, *dM);              // row count decided on the device
  if (static_cast<int>(blockIdx.y) * kTM >= M) return;
  // split K: block z sums k in [z kchunk, (z+1) kchunk) into plane z of C
  int k_begin = 0, k_end = K;
  if (kchunk > 0) {
    k_begin = static_cast<int>(blockIdx.z) * kchunk;
    k_end = min(K, k_begin + kchunk);
    C += static_cast<long>(blockIdx.z) * M * ldc;
  }
  __shared__ float As[kTM * kLdsK];
  __shared__ float Bs[kTN * kLdsK];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;

  // FP32 path accumulators: thread (tr, tc) owns rows tr*4.., cols tc*4..
  float acc[4][4];
  // MFMA path accumulators: wave w owns quadrant (w/2, w%2), 2x2 tiles of 16x16
  f32x4 macc[2][2];
  for (int i = 0; i < 4; ++i)
    for (int jx = 0; jx < 4; ++jx) acc[i][jx] = 0.f;
  for (int i = 0; i < 2; ++i)
    for (int jx = 0; jx < 2; ++jx) macc[i][jx] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int wave = tid >> 6, lane = tid & 63;
  // stage A (64 x 32) and B^T (64 x 32) as FP32: element q = tid + 256 i of a
  // tile, the unit-stride index running fastest across threads (coalesced);
  // the loads of the next K step are issued before the current one is used
  constexpr int kQ = kTM * kTK / 256;
  float va[kQ], vb[kQ];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = tid + 256 * i;
      const int r = (sak == 1) ? q / kTK : q % kTM;
      const int k = (sak == 1) ? q % kTK : q / kTM;
      const int gr = m0 + r, gk = k0 + k;
      va[i] = (gr < M && gk < k_end) ? A[gr * sar + gk * sak] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = tid + 256 * i;
      const int r = (sbk == 1) ? q / kTK : q % kTN;
      const int k = (sbk == 1) ? q % kTK : q / kTN;
      const int gn = n0 + r, gk = k0 + k;
      vb[i] = (gn < N && gk < k_end) ? B[gn * sbn + gk * sbk] : 0.f;
    }
  };
  if (k_begin < k_end) fetch(k_begin);
  for (int k0 = k_begin; k0 < k_end; k0 += kTK) {
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = tid + 256 * i;
      const int r = (sak == 1) ? q / kTK : q % kTM;
      const int k = (sak == 1) ? q % kTK : q / kTM;
      As[r * kLdsK + k] = va[i];
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = tid + 256 * i;
      const int r = (sbk == 1) ? q / kTK : q % kTN;
      const int k = (sbk == 1) ? q % kTK : q / kTN;
      Bs[r * kLdsK + k] = vb[i];
    }
    __syncthreads();
    if (k0 + kTK < k_end) fetch(k0 + kTK);
    if (MODE == kF32) {
      const int tr = tid >> 4, tc = tid & 15;
      for (int k = 0; k < kTK; ++k) {
        float a[4], b[4];
        for (int i = 0; i < 4; ++i) a[i] = As[(tr * 4 + i) * kLdsK + k];
        for (int i = 0; i < 4; ++i) b[i] = Bs[(tc * 4 + i) * kLdsK + k];
        for (int i = 0; i < 4; ++i)
          for (int jx = 0; jx < 4; ++jx) acc[i][jx] = __builtin_fmaf(a[i], b[jx], acc[i][jx]);
      }
    } else {
      // operand fragments: lane l -> row/col l%16, k = 8*(l/16) + i
      const int rq = (wave >> 1) * 32, cq = (wave & 1) * 32;
      const int fr = lane & 15, fk = 8 * (lane >> 4);
      bf16x8 bfrag[2];
      for (int tn = 0; tn < 2; ++tn) {
        const float* bp = &Bs[(cq + tn * 16 + fr) * kLdsK + fk];
        for (int i = 0; i < 8; ++i) bfrag[tn][i] = to_bf16(bp[i]);
      }
      for (int tm = 0; tm < 2; ++tm) {
        const float* ap = &As[(rq + tm * 16 + fr) * kLdsK + fk];
        bf16x8 a1, a2, a3;
        for (int i = 0; i < 8; ++i) {
          const float x = ap[i];
          const __bf16 h = to_bf16(x);
          a1[i] = h;
          if (MODE == kBF16S) {
            const float r1 = x - from_bf16(h);
            const __bf16 h2 = to_bf16(r1);
            a2[i] = h2;
            a3[i] = to_bf16(r1 - from_bf16(h2));
          }
        }
        for (int tn = 0; tn < 2; ++tn) {
          if (MODE == kBF16S) {
            macc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, bfrag[tn], macc[tm][tn], 0, 0, 0);
            macc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bfrag[tn], macc[tm][tn], 0, 0, 0);
          }
          macc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bfrag[tn], macc[tm][tn], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // epilogue
  if (MODE == kF32) {
    const int tr = tid >> 4, tc = tid & 15;
    for (int i = 0; i < 4; ++i) {
      const int r = m0 + tr * 4 + i;
      if (r >= M) continue;
      for (int jx = 0; jx < 4; ++jx) {
        const int n = n0 + tc * 4 + jx;
        if (n >= N) continue;
        float z = acc[i][jx] + (bias ? bias[n] : 0.f);
        if (Z) Z[r * ldz + n] = z;
        const float h = act_fwd(act, z);
        if (Csplit) store_split(Csplit, plane, r * ldc + n, h);
        else C[r * ldc + n] = h;
      }
    }
  } else {
    // output fragment: lane l holds rows 4*(l/16)+i, col l%16 of its 16x16 tile
    const int rq = (wave >> 1) * 32, cq = (wave & 1) * 32;
    for (int tm = 0; tm < 2; ++tm)
      for (int tn = 0; tn < 2; ++tn)
        for (int i = 0; i < 4; ++i) {
          const int r = m0 + rq + tm * 16 + 4 * (lane >> 4) + i;
          const int n = n0 + cq + tn * 16 + (lane & 15);
          if (r >= M || n >= N) continue;
          float z = macc[tm][tn][i] + (bias ? bias[n] : 0.f);
          if (Z) Z[r * ldz + n] = z;
          const float h = act_fwd(act, z);
          if (Csplit) store_split(Csplit, plane, r * ldc + n, h);
          else C[r * ldc + n] = h;
        }
  }
}

static hipError_t gemm_grid(int mode, dim3 grid, int M, int N, int K, const float* A, long sar, long sak,
                            const float* B, long sbn, long sbk, const float* bias, int act, float* C,
                            long ldc, float* Z, long ldz, const int* gate, hipStream_t s, const int* dM,
                            __bf16* Csplit, long plane, int kchunk) {
  const dim3 block(256);
  if (mode == kF32)
    hipLaunchKernelGGL(k_gemm<kF32>, grid, block, 0, s, M, N, K, A, sar, sak, B, sbn, sbk, bias,
                       act, C, ldc, Z, ldz, gate, dM, Csplit, plane, kchunk);
  else if (mode == kBF16S)
    hipLaunchKernelGGL(k_gemm<kBF16S>, grid, block, 0, s, M, N, K, A, sar, sak, B, sbn, sbk, bias,
                       act, C, ldc, Z, ldz, gate, dM, Csplit, plane, kchunk);
  else
    hipLaunchKernelGGL(k_gemm<kBF16>, grid, block, 0, s, M, N, K, A, sar, sak, B, sbn, sbk, bias,
                       act, C, ldc, Z, ldz, gate, dM, Csplit, plane, kchunk);
  return hipGetLastError();
}

hipError_t launch_gemm(int mode, int M, int N, int K, const float* A, long sar, long sak,
                       const float* B, long sbn, long sbk, const float* bias, int act, float* C,
                       long ldc, float* Z, long ldz, const int* gate, hipStream_t s, const int* dM,
                       __bf16* Csplit, long plane) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM);
  return gemm_grid(mode, grid, M, N, K, A, sar, sak, B, sbn, sbk, bias, act, C, ldc, Z, ldz, gate, s, dM,
                   Csplit, plane, 0);
}

// out[i] = sum_z part[z n + i], z = 0..S-1 in order
__global__ void k_sum_planes(int S, long n, const float* __restrict__ part, float* __restrict__ out) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float t = 0.f;
  for (int z = 0; z < S; ++z) t += part[z * n + i];
  out[i] = t;
}

hipError_t launch_gemm_splitk(int mode, int M, int N, int K, const float* A, long sar, long sak,
                              const float* B, long sbn, long sbk, float* C, float* work, long work_elems,
                              hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tiles = ((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM);
  int S = 1;
  // split the reduction until about four workgroups per CU run (chunks of at
  // least 256 rows of K)
  while (tiles * S < 1024 && K / (S * 2) >= 256 && static_cast<long>(2 * S) * M * N <= work_elems) S *= 2;
  if (S == 1)
    return launch_gemm(mode, M, N, K, A, sar, sak, B, sbn, sbk, nullptr, kActNone, C, N, nullptr, 0,
                       nullptr, s);
  const int kchunk = ((K + S - 1) / S + kTK - 1) / kTK * kTK;
  const dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM, (K + kchunk - 1) / kchunk);
  hipError_t e = gemm_grid(mode, grid, M, N, K, A, sar, sak, B, sbn, sbk, nullptr, kActNone, work, N,
                           nullptr, 0, nullptr, s, nullptr, nullptr, 0, kchunk);
  if (e != hipSuccess) return e;
  const long n = static_cast<long>(M) * N;
  hipLaunchKernelGGL(k_sum_planes, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<int>(grid.z), n, work, C);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense layer on split-bfloat16 activations (the emulator's layers 2..L):
//   C = act( (A_hi + A_mid + A_lo) W + b ),  W given transposed as bfloat16
//   Wt[N][K], activations as three bfloat16 planes [M][K] (K contiguous).
// Each wave computes a 32 x 32 block as 2 x 2 v_mfma_f32_16x16x32_bf16 tiles;
// operand fragments (8 consecutive k of one row / column) are 16-byte loads
// from L2, double-buffered in registers.  For every k-step of 32 the lo, mid
// and hi products are accumulated in that order, as in k_gemm<kBF16S>.
// Output: FP32 rows (C) or again three bfloat16 planes (Csplit).
// Requires K % 32 == 0 and M >= 1.
__global__ void __launch_bounds__(256)
k_dense_split(int M, int N, int K, const __bf16* __restrict__ A, long aplane, const __bf16* __restrict__ Wt,
              const float* __restrict__ bias, int act, float* __restrict__ C, __bf16* __restrict__ Csplit,
              long cplane, const int* __restrict__ gate, const int* __restrict__ dM) {
  if (gate && *gate == 0) return;
  if (dM) M = min(M, *dM);
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (m0 >= M) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rq = m0 + (wave >> 1) * 32, cq = n0 + (wave & 1) * 32;
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  // row / column of each fragment (clamped rows are computed and discarded)
  const __bf16* ap[2];
  const __bf16* bp[2];
  for (int t = 0; t < 2; ++t) {
    const int r = min(rq + t * 16 + fr, M - 1);
    ap[t] = A + static_cast<long>(r) * K + fk;
    const int cidx = min(cq + t * 16 + fr, N - 1);
    bp[t] = Wt + static_cast<long>(cidx) * K + fk;
  }
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int jx = 0; jx < 2; ++jx) acc[i][jx] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a_cur[2][3], b_cur[2], a_nxt[2][3], b_nxt[2];
  for (int t = 0; t < 2; ++t) {
    for (int sp = 0; sp < 3; ++sp) a_cur[t][sp] = *reinterpret_cast<const bf16x8*>(ap[t] + sp * aplane);
    b_cur[t] = *reinterpret_cast<const bf16x8*>(bp[t]);
  }
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bool more = k0 + 32 < K;
    if (more) {
      for (int t = 0; t < 2; ++t) {
        for (int sp = 0; sp < 3; ++sp)
          a_nxt[t][sp] = *reinterpret_cast<const bf16x8*>(ap[t] + sp * aplane + k0 + 32);
        b_nxt[t] = *reinterpret_cast<const bf16x8*>(bp[t] + k0 + 32);
      }
    }
    for (int tm = 0; tm < 2; ++tm)
      for (int tn = 0; tn < 2; ++tn) {
        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_cur[tm][2], b_cur[tn], acc[tm][tn], 0, 0, 0);
        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_cur[tm][1], b_cur[tn], acc[tm][tn], 0, 0, 0);
        acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_cur[tm][0], b_cur[tn], acc[tm][tn], 0, 0, 0);
      }
    if (more) {
      for (int t = 0; t < 2; ++t) {
        for (int sp = 0; sp < 3; ++sp) a_cur[t][sp] = a_nxt[t][sp];
        b_cur[t] = b_nxt[t];
      }
    }
  }
  for (int tm = 0; tm < 2; ++tm)
    for (int tn = 0; tn < 2; ++tn)
      for (int i = 0; i < 4; ++i) {
        const int r = rq + tm * 16 + 4 * (lane >> 4) + i;
        const int n = cq + tn * 16 + (lane & 15);
        if (r >= M || n >= N) continue;
        const float h = act_fwd(act, acc[tm][tn][i] + (bias ? bias[n] : 0.f));
        if (Csplit) store_split(Csplit, cplane, static_cast<long>(r) * N + n, h);
        else C[static_cast<long>(r) * N + n] = h;
      }
}

hipError_t launch_dense_split(int M, int N, int K, const __bf16* A, long aplane, const __bf16* Wt,
                              const float* bias, int act, float* C, __bf16* Csplit, long cplane,
                              const int* gate, const int* dM, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((N + 63) / 64, (M + 63) / 64), block(256);
  hipLaunchKernelGGL(k_dense_split, grid, block, 0, s, M, N, K, A, aplane, Wt, bias, act, C, Csplit, cplane,
                     gate, dM);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Emulator likelihood on fragment-major activations (frag_index): each
// operand load of a wave is one contiguous 1 KB read.  Activations travel as
// three such planes (hi, mid, lo); the transposed weights W^T[N][K] use the
// same layout (rows = output columns).  Row counts are padded to a multiple
// of 16; padded rows hold unspecified values and never reach an output.

// One dense layer on split activations: one wave per workgroup computes a
// 16 x 32 output block as two 16 x 16 MFMA tiles, k in steps of 32 with the
// loads of the next two steps in flight.  WS = 1: bfloat16 weights, products
// lo, mid, hi in that order (as k_dense_split); WS = 3 (the first layer, whose
// FP32 weights are split like the activations): the nine products of the
// activation and weight terms, smallest first.  Hidden layers: act(z) as three fragment-major planes of
// width N (transposed through LDS, 16-byte stores).  CHI2: the output layer;
// instead of storing y = z, every row's sum over the block's 32 columns of
// ((y - data) isig)^2 (FP64) goes to part[block column * pstride + r].
template <bool CHI2, int WS>
__global__ void __launch_bounds__(64)
k_dense_frag(int M, int N, int K, const __bf16* __restrict__ A, long aplane, const __bf16* __restrict__ Wf,
             long wplane, const float* __restrict__ bias, int act, __bf16* __restrict__ out, long cplane,
             const double* __restrict__ data, const double* __restrict__ isig, double* __restrict__ part,
             long pstride, const int* __restrict__ gate, const int* __restrict__ dM) {
  if (gate && *gate == 0) return;
  if (dM) M = min(M, *dM);
  const int nbc = N >> 5;
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int rb = bx / nbc, cb = bx - rb * nbc;
  if (rb * 16 >= M) return;
  const int lane = threadIdx.x;
  const int S = K >> 5;
  const __bf16* ap = A + static_cast<long>(rb) * S * 512 + lane * 8;
  const __bf16* bp0 = Wf + static_cast<long>(2 * cb) * S * 512 + lane * 8;
  const __bf16* bp1 = bp0 + static_cast<long>(S) * 512;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  bf16x8 a0[3], a1[3], a2[3], b0[2 * WS], b1[2 * WS], b2[2 * WS];
  auto load = [&](int s, bf16x8* a, bf16x8* b) {
    const long o = static_cast<long>(s) * 512;
    a[0] = *reinterpret_cast<const bf16x8*>(ap + o);
    a[1] = *reinterpret_cast<const bf16x8*>(ap + aplane + o);
    a[2] = *reinterpret_cast<const bf16x8*>(ap + 2 * aplane + o);
#pragma unroll
    for (int q = 0; q < WS; ++q) {
      b[2 * q] = *reinterpret_cast<const bf16x8*>(bp0 + q * wplane + o);
      b[2 * q + 1] = *reinterpret_cast<const bf16x8*>(bp1 + q * wplane + o);
    }
  };
  auto step = [&](const bf16x8* a, const bf16x8* b) {
    // term pairs (activation pa, weight pb) by decreasing pa + pb, then pa
#pragma unroll
    for (int sum = 2 + WS - 1; sum >= 0; --sum)
#pragma unroll
      for (int pa = 2; pa >= 0; --pa) {
        const int pb = sum - pa;
        if (pb < 0 || pb >= WS) continue;
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pa], b[2 * pb], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pa], b[2 * pb + 1], acc1, 0, 0, 0);
      }
  };
  load(0, a0, b0);
  if (S > 1) load(1, a1, b1);
  for (int s = 0; s < S; s += 3) {
    if (s + 2 < S) load(s + 2, a2, b2);
    step(a0, b0);
    if (s + 1 >= S) break;
    if (s + 3 < S) load(s + 3, a0, b0);
    step(a1, b1);
    if (s + 2 >= S) break;
    if (s + 4 < S) load(s + 4, a1, b1);
    step(a2, b2);
  }
  // output fragment: lane l holds rows 4 (l/16) + i, column l % 16 of each tile
  const int n0 = cb * 32 + (lane & 15);
  if (CHI2) {
    const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
    const double d0 = data[n0], d1 = data[n0 + 16], s0 = isig[n0], s1 = isig[n0 + 16];
    for (int i = 0; i < 4; ++i) {
      const double e0 = (static_cast<double>(acc0[i] + bz0) - d0) * s0;
      const double e1 = (static_cast<double>(acc1[i] + bz1) - d1) * s1;
      double t = e0 * e0 + e1 * e1;
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o);
      const int r = rb * 16 + 4 * (lane >> 4) + i;
      if ((lane & 15) == 0 && r < M) part[static_cast<long>(cb) * pstride + r] = t;
    }
  } else {
    __shared__ __attribute__((aligned(16))) __bf16 tile[3][16][32 + 8];
    const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
    for (int i = 0; i < 4; ++i) {
      const int rr = 4 * (lane >> 4) + i;
      for (int t = 0; t < 2; ++t) {
        const float x = act_fwd(act, (t ? acc1[i] : acc0[i]) + (t ? bz1 : bz0));
        const __bf16 h = to_bf16(x);
        const float r1 = x - from_bf16(h);
        const __bf16 md = to_bf16(r1);
        tile[0][rr][t * 16 + (lane & 15)] = h;
        tile[1][rr][t * 16 + (lane & 15)] = md;
        tile[2][rr][t * 16 + (lane & 15)] = to_bf16(r1 - from_bf16(md));
      }
    }
    __syncthreads();
    const long o = (static_cast<long>(rb) * nbc + cb) * 512 + lane * 8;
    const int rr = lane & 15, g = lane >> 4;
    for (int p = 0; p < 3; ++p)
      *reinterpret_cast<bf16x8*>(out + p * cplane + o) = *reinterpret_cast<const bf16x8*>(&tile[p][rr][8 * g]);
  }
}

// The same layer for many rows: one wave per 32 x 64 output block (two row
// blocks of 16, four column tiles of 16), single-term weights (WS = 1).  Per
// K step of 32 the wave loads six activation fragments and four weight
// fragments (10 KB) for 24 MFMAs, twice the work per loaded byte of the 16 x 32
// block; every 16 x 16 tile accumulates its products in the same order as
// k_dense_frag, so the outputs are identical.  rows16: row blocks of 16 that
// exist (the second row block of the last wave may not).
template <bool CHI2>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_dense_frag_w(int M, int N, int K, const __bf16* __restrict__ A, long aplane, const __bf16* __restrict__ Wf,
               const float* __restrict__ bias, int act, __bf16* __restrict__ out, long cplane,
               const double* __restrict__ data, const double* __restrict__ isig, double* __restrict__ part,
               long pstride, const int* __restrict__ gate, const int* __restrict__ dM) {
  if (gate && *gate == 0) return;
  if (dM) M = min(M, *dM);
  const int nbw = N >> 6;
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int rw = bx / nbw, cw = bx - rw * nbw;
  if (rw * 32 >= M) return;
  const bool two = rw * 32 + 16 < M;   // second row block present
  const int lane = threadIdx.x;
  const int S = K >> 5;
  const __bf16* ap0 = A + static_cast<long>(2 * rw) * S * 512 + lane * 8;
  const __bf16* ap1 = ap0 + static_cast<long>(S) * 512;
  const __bf16* bp = Wf + static_cast<long>(4 * cw) * S * 512 + lane * 8;
  const long bstep = static_cast<long>(S) * 512;
  f32x4 acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a0[2][3], a1[2][3], a2[2][3], b0[4], b1[4], b2[4];
  auto load = [&](int s, bf16x8 (&a)[2][3], bf16x8 (&b)[4]) {
    const long o = static_cast<long>(s) * 512;
#pragma unroll
    for (int p = 0; p < 3; ++p) a[0][p] = *reinterpret_cast<const bf16x8*>(ap0 + p * aplane + o);
#pragma unroll
    for (int p = 0; p < 3; ++p)
      a[1][p] = two ? *reinterpret_cast<const bf16x8*>(ap1 + p * aplane + o) : a[0][p];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const bf16x8*>(bp + j * bstep + o);
  };
  auto step = [&](const bf16x8 (&a)[2][3], const bf16x8 (&b)[4]) {
    // activation terms by decreasing pa (the weight has one term)
#pragma unroll
    for (int pa = 2; pa >= 0; --pa)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r][pa], b[j], acc[r][j], 0, 0, 0);
  };
  // two steps of loads in flight
  load(0, a0, b0);
  if (S > 1) load(1, a1, b1);
  for (int s = 0; s < S; s += 3) {
    if (s + 2 < S) load(s + 2, a2, b2);
    step(a0, b0);
    if (s + 1 >= S) break;
    if (s + 3 < S) load(s + 3, a0, b0);
    step(a1, b1);
    if (s + 2 >= S) break;
    if (s + 4 < S) load(s + 4, a1, b1);
    step(a2, b2);
  }
  const int nl = lane & 15;
  if (CHI2) {
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      const int n0 = cw * 64 + c2 * 32 + nl;
      const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
      const double d0 = data[n0], d1 = data[n0 + 16], s0 = isig[n0], s1 = isig[n0 + 16];
#pragma unroll
      for (int r = 0; r < 2; ++r)
        for (int i = 0; i < 4; ++i) {
          const double e0 = (static_cast<double>(acc[r][2 * c2][i] + bz0) - d0) * s0;
          const double e1 = (static_cast<double>(acc[r][2 * c2 + 1][i] + bz1) - d1) * s1;
          double t = e0 * e0 + e1 * e1;
          for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o);
          const int row = (2 * rw + r) * 16 + 4 * (lane >> 4) + i;
          if (nl == 0 && row < M) part[static_cast<long>(2 * cw + c2) * pstride + row] = t;
        }
    }
  } else {
    __shared__ __attribute__((aligned(16))) __bf16 tile[3][16][32 + 8];
    const int nbc = N >> 5;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (r == 1 && !two) break;
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) {
        const int n0 = cw * 64 + c2 * 32 + nl;
        const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
        for (int i = 0; i < 4; ++i) {
          const int rr = 4 * (lane >> 4) + i;
          for (int t = 0; t < 2; ++t) {
            const float x = act_fwd(act, acc[r][2 * c2 + t][i] + (t ? bz1 : bz0));
            const __bf16 h = to_bf16(x);
            const float r1 = x - from_bf16(h);
            const __bf16 md = to_bf16(r1);
            tile[0][rr][t * 16 + nl] = h;
            tile[1][rr][t * 16 + nl] = md;
            tile[2][rr][t * 16 + nl] = to_bf16(r1 - from_bf16(md));
          }
        }
        __syncthreads();
        const long o = (static_cast<long>(2 * rw + r) * nbc + 2 * cw + c2) * 512 + lane * 8;
        const int rr = lane & 15, g = lane >> 4;
        for (int p = 0; p < 3; ++p)
          *reinterpret_cast<bf16x8*>(out + p * cplane + o) = *reinterpret_cast<const bf16x8*>(&tile[p][rr][8 * g]);
        __syncthreads();
      }
    }
  }
}

// The same layer for many rows on (64 RW) x 128 output tiles per workgroup
// (four waves; wave w: row blocks RW w .. RW w + RW - 1 of the tile, all eight
// column tiles), single-term weights.  Per K step of 32 the workgroup copies
// its 12 RW activation fragments and 8 weight fragments into one of two LDS
// buffers (one 16-byte load per thread and fragment row of the copy, issued
// two steps ahead) while the waves run 24 RW MFMAs each out of the other;
// every 16 x 16 tile sums its products in the same order as k_dense_frag
// (identical outputs).
template <int RW>
constexpr int tile_frags() { return 12 * RW + 8; }

template <bool CHI2, int RW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_dense_frag_t(int M, int N, int K, const __bf16* __restrict__ A, long aplane, const __bf16* __restrict__ Wf,
               const float* __restrict__ bias, int act, __bf16* __restrict__ out, long cplane,
               const double* __restrict__ data, const double* __restrict__ isig, double* __restrict__ part,
               long pstride, const int* __restrict__ gate, const int* __restrict__ dM) {
  constexpr int F = tile_frags<RW>(), NA = 12 * RW, Q = F / 4;   // fragments per step; 16-byte loads per thread
  constexpr int TR = 4 * RW;                                      // row blocks per tile
  __shared__ __attribute__((aligned(16))) bf16x8 lds[2][F * 64];
  if (gate && *gate == 0) return;
  if (dM) M = min(M, *dM);
  const int nbt = N >> 7;
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int rt = bx / nbt, ct = bx - rt * nbt;
  if (rt * 16 * TR >= M) return;
  const int nrb = (M + 15) >> 4;                 // row blocks that exist
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int S = K >> 5;
  // copy assignment: chunk c = tid + 256 i (i < Q) of the 64 F 16-byte chunks
  // of a step; fragment f = c / 64: activation row block f / 3, plane f % 3
  // for f < 12 RW, weight column tile f - 12 RW after that
  const bf16x8* gsrc[Q];
  bool have[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int c = tid + 256 * i, f = c >> 6, within = (c & 63) * 8;
    if (f < NA) {
      const int rbl = f / 3, p = f - 3 * rbl, rbg = rt * TR + rbl;
      have[i] = rbg < nrb;
      gsrc[i] = reinterpret_cast<const bf16x8*>(A + p * aplane + static_cast<long>(min(rbg, nrb - 1)) * S * 512 +
                                                within);
    } else {
      have[i] = true;
      gsrc[i] = reinterpret_cast<const bf16x8*>(Wf + static_cast<long>(ct * 8 + f - NA) * S * 512 + within);
    }
  }
  bf16x8 st0[Q], st1[Q];
  auto fetch = [&](int s, bf16x8 (&st)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) st[i] = have[i] ? gsrc[i][s * 64] : bf16x8{};
  };
  auto put = [&](int buf, const bf16x8 (&st)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) lds[buf][tid + 256 * i] = st[i];
  };
  f32x4 acc[RW][8];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int buf) {
    bf16x8 a[RW][3], b[8];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int p = 0; p < 3; ++p) a[r][p] = lds[buf][((RW * wv + r) * 3 + p) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = lds[buf][(NA + j) * 64 + lane];
    // activation terms by decreasing pa (the weight has one term)
#pragma unroll
    for (int pa = 2; pa >= 0; --pa)
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r][pa], b[j], acc[r][j], 0, 0, 0);
  };
  // step k's loads go to st[k & 1]; step s + 2 is fetched before step s runs
  fetch(0, st0);
  if (S > 1) fetch(1, st1);
  put(0, st0);
  __syncthreads();
  for (int s = 0; s < S; s += 2) {
    if (s + 2 < S) fetch(s + 2, st0);
    compute(0);
    if (s + 1 >= S) break;
    put(1, st1);
    __syncthreads();
    if (s + 3 < S) fetch(s + 3, st1);
    compute(1);
    if (s + 2 < S) put(0, st0);
    __syncthreads();
  }
  // the epilogue reuses the LDS: every wave is past its last reads
  __syncthreads();
  const int nl = lane & 15;
  if (CHI2) {
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const int n0 = ct * 128 + c2 * 32 + nl;
      const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
      const double d0 = data[n0], d1 = data[n0 + 16], s0 = isig[n0], s1 = isig[n0 + 16];
#pragma unroll
      for (int r = 0; r < RW; ++r)
        for (int i = 0; i < 4; ++i) {
          const double e0 = (static_cast<double>(acc[r][2 * c2][i] + bz0) - d0) * s0;
          const double e1 = (static_cast<double>(acc[r][2 * c2 + 1][i] + bz1) - d1) * s1;
          double t = e0 * e0 + e1 * e1;
          for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o);
          const int row = (rt * TR + RW * wv + r) * 16 + 4 * (lane >> 4) + i;
          if (nl == 0 && row < M) part[static_cast<long>(ct * 4 + c2) * pstride + row] = t;
        }
    }
  } else {
    // per wave: a 3 x 16 x 40 bf16 transposition tile in the (now idle) LDS
    __bf16 (*tile)[16][40] =
        reinterpret_cast<__bf16 (*)[16][40]>(reinterpret_cast<unsigned char*>(&lds[0][0]) + wv * (3 * 16 * 40 * 2));
    const int nbc = N >> 5;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int rbg = rt * TR + RW * wv + r;
      if (rbg >= nrb) break;
#pragma unroll
      for (int c2 = 0; c2 < 4; ++c2) {
        const int n0 = ct * 128 + c2 * 32 + nl;
        const float bz0 = bias ? bias[n0] : 0.f, bz1 = bias ? bias[n0 + 16] : 0.f;
        for (int i = 0; i < 4; ++i) {
          const int rr = 4 * (lane >> 4) + i;
          for (int t = 0; t < 2; ++t) {
            const float x = act_fwd(act, acc[r][2 * c2 + t][i] + (t ? bz1 : bz0));
            const __bf16 h = to_bf16(x);
            const float r1 = x - from_bf16(h);
            const __bf16 md = to_bf16(r1);
            tile[0][rr][t * 16 + nl] = h;
            tile[1][rr][t * 16 + nl] = md;
            tile[2][rr][t * 16 + nl] = to_bf16(r1 - from_bf16(md));
          }
        }
        // only this wave reads its tile (no workgroup barrier: waves leave the
        // loop at different row blocks); the fence completes its LDS writes
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        const long o = (static_cast<long>(rbg) * nbc + ct * 4 + c2) * 512 + lane * 8;
        const int rr = lane & 15, g = lane >> 4;
        for (int p = 0; p < 3; ++p)
          *reinterpret_cast<bf16x8*>(out + p * cplane + o) = *reinterpret_cast<const bf16x8*>(&tile[p][rr][8 * g]);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      }
    }
  }
}

// logL[r] = -1/2 sum_q part[q pstride + r] (q ascending); NaN -> -inf.
__global__ void k_chi2_sum(int M, int nb, const double* __restrict__ part, long pstride, double* __restrict__ logL,
                           const int* __restrict__ gate, const int* __restrict__ dM) {
  if (gate && *gate == 0) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M || (dM && r >= *dM)) return;
  // loads in groups of eight ahead of the (in-order) additions
  double t = 0.0;
  for (int q0 = 0; q0 < nb; q0 += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[min(q0 + j, nb - 1) * pstride + r];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (q0 + j < nb) t += v[j];
  }
  const double v = -0.5 * t;
  logL[r] = isnan(v) ? -INFINITY : v;
}


bool emu_frag_eligible(const NetDev& net, int mode_first, int mode_rest) {
  if (mode_first != kF32 || mode_rest != kBF16S || net.n_layers < 2 || net.widths[0] > 32) return false;
  for (int l = 1; l <= net.n_layers; ++l)
    if (net.widths[l] % 32 != 0) return false;
  for (int l = 0; l < net.n_layers; ++l)
    if (!net.Wf[l]) return false;
  return true;
}

long emu_frag_plane(long M, int max_width) { return (M + 15) / 16 * 16 * max_width; }

hipError_t emu_forward_logL(const NetDev& net, int M, const __bf16* Xf, long xplane, __bf16* P0, __bf16* P1,
                            double* part, const double* data, const double* isig, double* logL, const int* gate,
                            const int* dM, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const long plane = emu_frag_plane(M, net.max_width);
  const int L = net.n_layers;
  const int rbs = (M + 15) / 16;
  const __bf16* in = Xf;
  long inplane = xplane;
  __bf16* out = P0;
  for (int l = 0; l < L; ++l) {
    const int K = l == 0 ? 32 : net.widths[l], N = net.widths[l + 1];
    const dim3 grid(static_cast<unsigned>(rbs * (N / 32)));
    if (l == 0 && net.w0_planes == 1) {
      // bfloat16 first-layer weights: the mid and lo weight planes are zero
      hipLaunchKernelGGL((k_dense_frag<false, 1>), grid, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[0], 0L,
                         net.b[0], net.act, out, plane, nullptr, nullptr, nullptr, 0L, gate, dM);
    } else if (l == 0) {
      hipLaunchKernelGGL((k_dense_frag<false, 3>), grid, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[0],
                         static_cast<long>(N) * 32, net.b[0], net.act, out, plane, nullptr, nullptr, nullptr, 0L,
                         gate, dM);
    } else if (l == L - 1 && N % 128 == 0 && ((M + 127) / 128) * (N / 128) >= kFragTileMin) {
      // many rows, output layer: 128 x 128 tiles per workgroup, operands in LDS
      const dim3 gt(static_cast<unsigned>(((M + 127) / 128) * (N / 128)));
      hipLaunchKernelGGL((k_dense_frag_t<true, 2>), gt, dim3(256), 0, s, M, N, K, in, inplane, net.Wf[l], net.b[l],
                         kActNone, nullptr, 0L, data, isig, part, static_cast<long>(M), gate, dM);
    } else if (l < L - 1 && N % 128 == 0 && ((M + 63) / 64) * (N / 128) >= kFragTileMin) {
      // many rows, hidden layer: 64 x 128 tiles per workgroup, operands in LDS
      const dim3 gt(static_cast<unsigned>(((M + 63) / 64) * (N / 128)));
      hipLaunchKernelGGL((k_dense_frag_t<false, 1>), gt, dim3(256), 0, s, M, N, K, in, inplane, net.Wf[l], net.b[l],
                         net.act, out, plane, nullptr, nullptr, nullptr, 0L, gate, dM);
    } else if (M >= kFragWideRows && N % 64 == 0) {
      // many rows: 32 x 64 blocks per wave (the same sums, more reuse per load)
      const dim3 gw(static_cast<unsigned>(((M + 31) / 32) * (N / 64)));
      if (l < L - 1)
        hipLaunchKernelGGL((k_dense_frag_w<false>), gw, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[l], net.b[l],
                           net.act, out, plane, nullptr, nullptr, nullptr, 0L, gate, dM);
      else
        hipLaunchKernelGGL((k_dense_frag_w<true>), gw, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[l], net.b[l],
                           kActNone, nullptr, 0L, data, isig, part, static_cast<long>(M), gate, dM);
    } else if (l < L - 1) {
      hipLaunchKernelGGL((k_dense_frag<false, 1>), grid, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[l], 0L,
                         net.b[l], net.act, out, plane, nullptr, nullptr, nullptr, 0L, gate, dM);
    } else {
      hipLaunchKernelGGL((k_dense_frag<true, 1>), grid, dim3(64), 0, s, M, N, K, in, inplane, net.Wf[l], 0L,
                         net.b[l], kActNone, nullptr, 0L, data, isig, part, static_cast<long>(M), gate, dM);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (l < L - 1) {
      in = out;
      inplane = plane;
      out = (out == P0) ? P1 : P0;
    }
  }
  if (!logL) return hipSuccess;   // the caller sums the partials (launch_scatter)
  hipLaunchKernelGGL(k_chi2_sum, dim3((M + 255) / 256), dim3(256), 0, s, M, net.widths[L] / 32, part,
                     static_cast<long>(M), logL, gate, dM);
  return hipGetLastError();
}

void frag_layout_host(const float* Wt, int N, int K, __bf16* out) {
  for (int n = 0; n < N; ++n)
    for (int k = 0; k < K; ++k) out[frag_index(n, k, K)] = static_cast<__bf16>(Wt[static_cast<long>(n) * K + k]);
}

void frag_split_host(const float* Wt, int N, int K0, __bf16* out) {
  const long plane = static_cast<long>(N) * 32;
  for (long q = 0; q < 3 * plane; ++q) out[q] = static_cast<__bf16>(0.f);
  for (int n = 0; n < N; ++n)
    for (int k = 0; k < K0; ++k) {
      const float x = Wt[static_cast<long>(n) * K0 + k];
      const __bf16 h = static_cast<__bf16>(x);
      const float r1 = x - static_cast<float>(h);
      const __bf16 m = static_cast<__bf16>(r1);
      const long idx = frag_index(n, k, 32);
      out[idx] = h;
      out[plane + idx] = m;
      out[2 * plane + idx] = static_cast<__bf16>(r1 - static_cast<float>(m));
    }
}

// ---------------------------------------------------------------------------
// Elementwise pieces of the backward pass and the diagonal chi^2.

// dZ = dH * act'(Z)
__global__ void k_act_bwd(long n, int act, const float* __restrict__ Z, const float* __restrict__ dH,
                          float* __restrict__ dZ) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float z = Z[i];
  float g = 1.f;
  if (act == kActTanh) {
    const float t = tanhf(z);
    g = 1.f - t * t;
  } else if (act == kActSilu) {
    const float sg = 1.f / (1.f + expf(-z));
    g = sg * (1.f + z * (1.f - sg));
  }
  dZ[i] = dH[i] * g;
}

hipError_t launch_act_bwd(long n, int act, const float* Z, const float* dH, float* dZ, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_act_bwd, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, n, act,
                     Z, dH, dZ);
  return hipGetLastError();
}

// db[n] = sum_r dZ[r, n] in a fixed order.  With a workspace: chunks of 256
// rows, each summed by 4 row groups of one workgroup (64 columns per
// workgroup, coalesced), then the chunk partials in chunk order.
__global__ void k_colsum(int M, int N, const float* __restrict__ dZ, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int r = 0; r < M; ++r) s += dZ[static_cast<long>(r) * N + n];
  db[n] = s;
}

__global__ void __launch_bounds__(256)
k_colsum_part(int M, int N, const float* __restrict__ dZ, float* __restrict__ part) {
  __shared__ float red[256];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int r0 = blockIdx.y * 256, r1 = min(M, r0 + 256);
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int r = r0 + g; r < r1; r += 4) s += dZ[static_cast<long>(r) * N + n];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && n < N)
    part[static_cast<long>(blockIdx.y) * N + n] = ((red[c] + red[64 + c]) + red[128 + c]) + red[192 + c];
}

hipError_t launch_colsum(int M, int N, const float* dZ, float* db, hipStream_t s, float* work,
                         long work_elems) {
  if (N <= 0) return hipSuccess;
  const int chunks = (M + 255) / 256;
  if (work && chunks > 1 && static_cast<long>(chunks) * N <= work_elems) {
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, chunks), dim3(256), 0, s, M, N, dZ, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_planes, dim3((N + 255) / 256), dim3(256), 0, s, chunks, static_cast<long>(N),
                       work, db);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, M, N, dZ, db);
  return hipGetLastError();
}

// logL[r] = -1/2 sum_i ((y_ri - data_i) * isig_i)^2 in FP64; rows with flag 0 get -inf.
__global__ void __launch_bounds__(64)
k_chi2(int M, int N, const float* __restrict__ Y, const double* __restrict__ data,
       const double* __restrict__ isig, const int* __restrict__ flag, double* __restrict__ logL,
       const int* __restrict__ gate, const int* __restrict__ dM) {
  if (gate && *gate == 0) return;
  const int r = blockIdx.x;
  if (r >= M || (dM && r >= *dM)) return;
  const int lane = threadIdx.x;
  if (flag && flag[r] == 0) {
    if (lane == 0) logL[r] = -INFINITY;
    return;
  }
  double s = 0.0;
  for (int i = lane; i < N; i += 64) {
    const double e = (static_cast<double>(Y[static_cast<long>(r) * N + i]) - data[i]) * isig[i];
    s += e * e;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (lane == 0) {
    const double v = -0.5 * s;
    logL[r] = isnan(v) ? -INFINITY : v;
  }
}

hipError_t launch_chi2(int M, int N, const float* Y, const double* data, const double* isig,
                       const int* flag, double* logL, const int* gate, hipStream_t s, const int* dM) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chi2, dim3(M), dim3(64), 0, s, M, N, Y, data, isig, flag, logL, gate, dM);
  return hipGetLastError();
}

}  // namespace ns

namespace ns {

hipError_t net_forward(const NetDev& net, int mode_first, int mode_rest, int M, const float* X,
                       float* H0, float* H1, float* Y, const int* gate, hipStream_t s, const int* dM) {
  bool split = mode_rest == kBF16S && net.n_layers > 1;
  for (int l = 1; l < net.n_layers; ++l) split = split && net.Wb[l] != nullptr;
  if (split) {
    // first layer in FP32 written as split planes, then split-activation MFMA layers
    const long plane = static_cast<long>(M) * net.max_width;
    __bf16* P0 = reinterpret_cast<__bf16*>(H0);
    __bf16* P1 = reinterpret_cast<__bf16*>(H1);
    hipError_t e = launch_gemm(mode_first, M, net.widths[1], net.widths[0], X, net.widths[0], 1, net.Wt[0],
                               net.w_rowmajor ? 1 : net.widths[0], net.w_rowmajor ? net.widths[1] : 1,
                               net.b[0], net.n_layers > 1 ? net.act : kActNone, nullptr, net.widths[1],
                               nullptr, 0, gate, s, dM, net.n_layers > 1 ? P0 : nullptr, plane);
    if (e != hipSuccess || net.n_layers == 1) return e;
    __bf16* in = P0;
    __bf16* out = P1;
    for (int l = 1; l < net.n_layers; ++l) {
      const bool last = (l == net.n_layers - 1);
      e = launch_dense_split(M, net.widths[l + 1], net.widths[l], in, plane, net.Wb[l], net.b[l],
                             last ? kActNone : net.act, last ? Y : nullptr, last ? nullptr : out, plane,
                             gate, dM, s);
      if (e != hipSuccess) return e;
      std::swap(in, out);
    }
    return hipSuccess;
  }
  const float* in = X;
  long ldin = net.widths[0];
  for (int l = 0; l < net.n_layers; ++l) {
    const int K = net.widths[l], N = net.widths[l + 1];
    const bool last = (l == net.n_layers - 1);
    float* out = last ? Y : ((l % 2 == 0) ? H0 : H1);
    hipError_t e = launch_gemm(l == 0 ? mode_first : mode_rest, M, N, K, in, ldin, 1, net.Wt[l],
                               net.w_rowmajor ? 1 : K, net.w_rowmajor ? N : 1, net.b[l],
                               last ? kActNone : net.act, out, N, nullptr, 0, gate, s, dM);
    if (e != hipSuccess) return e;
    in = out;
    ldin = N;
  }
  return hipSuccess;
}

}  // namespace ns
