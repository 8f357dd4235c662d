// ns_gemm.hpp -- launchers of the dense-layer kernels (k_gemm.hip) and of the
// round-based slice sampler used with network likelihoods (k_slice_rounds.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "ns_device.hpp"

namespace ns {

enum GemmMode : int { kF32 = 0, kBF16S = 1, kBF16 = 2 };

// Fragment-major bfloat16 layout of a matrix with K columns (K % 32 == 0):
// blocks of 16 rows x 32 columns, block (r/16, k/32) at element
// ((r/16) (K/32) + k/32) 512; inside a block the eight columns 8g..8g+7 of row
// i are contiguous at element (i + 16 g) 8, so a block is exactly one
// 16x16x32 MFMA operand fragment (lane i + 16 g holds 16 bytes).
__host__ __device__ inline long frag_index(long r, int k, int K) {
  return ((r >> 4) * (K >> 5) + (k >> 5)) * 512 + ((r & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}
enum Act : int { kActNone = 0, kActTanh = 1, kActSilu = 2 };

// dM (may be null): device-side row count; rows at or beyond it are skipped.
// Csplit (may be null): write act(z) as three bfloat16 planes of `plane`
// elements (hi, mid, lo) instead of FP32 C.
hipError_t launch_gemm(int mode, int M, int N, int K, const float* A, long sar, long sak,
                       const float* B, long sbn, long sbk, const float* bias, int act, float* C,
                       long ldc, float* Z, long ldz, const int* gate, hipStream_t s,
                       const int* dM = nullptr, __bf16* Csplit = nullptr, long plane = 0);
hipError_t launch_dense_split(int M, int N, int K, const __bf16* A, long aplane, const __bf16* Wt,
                              const float* bias, int act, float* C, __bf16* Csplit, long cplane,
                              const int* gate, const int* dM, hipStream_t s);
hipError_t launch_act_bwd(long n, int act, const float* Z, const float* dH, float* dZ, hipStream_t s);
// work (may be null): workspace for the chunked column sum (>= ceil(M/256) * N floats)
hipError_t launch_colsum(int M, int N, const float* dZ, float* db, hipStream_t s, float* work = nullptr,
                         long work_elems = 0);
// C (M x N, ld N) = A B without bias or activation, splitting K across
// workgroups when the output has few tiles; partial products go to work
// (work_elems floats) and are added in a fixed order.
hipError_t launch_gemm_splitk(int mode, int M, int N, int K, const float* A, long sar, long sak,
                              const float* B, long sbn, long sbk, float* C, float* work, long work_elems,
                              hipStream_t s);
hipError_t launch_chi2(int M, int N, const float* Y, const double* data, const double* isig,
                       const int* flag, double* logL, const int* gate, hipStream_t s,
                       const int* dM = nullptr);

// A network held on the device: layer l maps widths[l] -> widths[l+1]; the
// weights are stored transposed (Wt_l: widths[l+1] x widths[l], FP32), or
// row major (widths[l] x widths[l+1]) when w_rowmajor is set.
struct NetDev {
  int n_layers;
  int widths[9];
  int act;              // hidden activation (output layer is linear)
  const float* Wt[8];
  const float* b[8];
  int max_width;
  int w_rowmajor;
  const __bf16* Wb[8];  // bfloat16 copies of Wt (layers >= 1) for the split-activation path
  const __bf16* Wf[8];  // the same in the fragment-major layout (emu_forward_logL); layer 0:
                        // hi, mid, lo planes of widths[1] x 32 (inputs padded with zeros)
  const float* Wq[8];   // FP32 W^T in 16 x 16 blocks for the FP32 MFMA (k_emu_chains, FP32
                        // layers); K padded with zeros to a multiple of 16
  int w0_planes;        // 1 when the first layer's weights are bfloat16 values (mid and lo
                        // planes zero: their products add exact zeros and are skipped), else 3
};

// Forward over M rows of X (M x widths[0]); H0/H1 ping-pong buffers of
// M x max_width floats; output Y (M x widths[L]).  mode_first applies to
// layer 0, mode_rest to the others.  With mode_rest == kBF16S and bfloat16
// weights present, hidden activations travel as three bfloat16 planes
// (3 M max_width bf16 = 1.5x the FP32 buffer: H0/H1 must hold that much).
hipError_t net_forward(const NetDev& net, int mode_first, int mode_rest, int M, const float* X,
                       float* H0, float* H1, float* Y, const int* gate, hipStream_t s,
                       const int* dM = nullptr);

// Emulator log-likelihood on fragment-major split activations (k_gemm.hip):
// every layer on bfloat16 MFMA with FP32 accumulation (the input and the
// first layer's weights split into three bfloat16 terms each, later layers'
// activations into three terms against bfloat16 weights), the diagonal chi^2
// (FP64) fused into the output layer.  Applies with layer 0 FP32, the others
// split bfloat16, at least two layers, widths[0] <= 32 and every other width
// a multiple of 32 (emu_frag_eligible).  Xf: the inputs as three
// fragment-major planes of (M rounded up to 16) x 32 (columns >= widths[0]
// zero), plane stride xplane.  P0/P1: three planes of emu_frag_plane(M,
// max_width) bfloat16 each; part: widths[L]/32 x M doubles (column block q of
// row r at q M + r).  With logL null the partials are left for the caller to
// sum (in ascending q, then -1/2, NaN -> -inf).
bool emu_frag_eligible(const NetDev& net, int mode_first, int mode_rest);
long emu_frag_plane(long M, int max_width);
hipError_t emu_forward_logL(const NetDev& net, int M, const __bf16* Xf, long xplane, __bf16* P0, __bf16* P1,
                            double* part, const double* data, const double* isig, double* logL, const int* gate,
                            const int* dM, hipStream_t s);
// Host: W^T (N x K FP32, N % 16 == 0, K % 32 == 0) -> fragment-major bfloat16.
void frag_layout_host(const float* Wt, int N, int K, __bf16* out);
// Host: W^T (N x K0 FP32, K0 <= 32) -> three fragment-major planes (hi, mid,
// lo) of N x 32, inputs K0..31 zero.
void frag_split_host(const float* Wt, int N, int K0, __bf16* out);

}  // namespace ns
