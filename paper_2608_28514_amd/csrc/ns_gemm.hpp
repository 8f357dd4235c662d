// ns_gemm.hpp -- launchers of the dense-layer kernels (k_gemm.hip) and of the
// round-based slice sampler used with network likelihoods (k_slice_rounds.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "ns_device.hpp"

namespace ns {

enum GemmMode : int { kF32 = 0, kBF16S = 1, kBF16 = 2 };
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
  const __bf16* Wf[8];  // the same in the fragment-major layout (emu_forward_logL)
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
// layer 0 in FP32, hidden layers and the output layer on bfloat16 MFMA, the
// diagonal chi^2 fused into the output layer.  Applies when layer 0 is FP32,
// the others split bfloat16, at least two layers, widths[0] <= 32 and every
// other width a multiple of 32 (emu_frag_eligible).  P0/P1: three planes of
// emu_frag_plane(M, max_width) bfloat16 each; part: M x widths[L]/32 doubles.
bool emu_frag_eligible(const NetDev& net, int mode_first, int mode_rest);
long emu_frag_plane(long M, int max_width);
hipError_t emu_forward_logL(const NetDev& net, int M, const float* X, __bf16* P0, __bf16* P1, double* part,
                            const double* data, const double* isig, double* logL, const int* gate,
                            const int* dM, hipStream_t s);
// Host: W^T (N x K FP32, N % 16 == 0, K % 32 == 0) -> fragment-major bfloat16.
void frag_layout_host(const float* Wt, int N, int K, __bf16* out);

}  // namespace ns
