// ns_rounds.hpp -- state and launchers of the round-based slice sampler
// (k_slice_rounds.hip), used when the likelihood is evaluated in batches.
#pragma once
#include <hip/hip_runtime.h>
#include "ns_internal.hpp"
#include "ns_gemm.hpp"

namespace ns {

enum Phase : int { kPhaseDir = 0, kPhaseStepout = 1, kPhaseShrink = 2, kPhaseDone = 3 };

template <typename T>
struct ChainState {
  T x[kMaxD];
  T v[kMaxD];
  double lx;
  T a0, b0, a, b, br_a, br_b;
  int it, phase, ka, kb, base, s0, hn, n_evals, n_oob, n_so, n_sh, label, seed_slot, n_scr;
};

struct RoundsParams {
  int m, d, T, P, n_iter, so_spec, sh_spec, max_stepout, max_shrink;
  double w;
  uint64_t seed;
  float lo_f[kMaxD];
  float span_f[kMaxD];
};

struct RoundBufs {
  void* cs;        // m chain states
  void* pts;       // rows x d, state precision
  float* xin;      // rows x d, network input theta
  int* flag;       // rows: 1 = in the box, evaluate
  double* rlogL;   // rows
  double* rthr;    // rows: the threshold the row is tested against
  int* sflag;      // rows: 1 = screened out by the surrogate (not evaluated)
  int* gate;       // per round: some chain still running
  long rows_cap;
  int gate_cap;
  float* H0;       // rows x max_width
  float* H1;
  float* Y;        // rows x out_width
  // Direct network evaluation (no row compaction pass): when xf_direct is set
  // the advance kernel also writes each chain's rows, split into three
  // bfloat16 terms, to compacted fragment-major planes (stride xf_plane);
  // crows[round] counts the compacted rows, cmap[c] is the chain of compacted
  // rows c P .. c P + P - 1.
  __bf16* xf_direct;
  long xf_plane;
  int* crows;      // gate_cap entries
  int* cmap;       // m entries
  // Direct rounds also leave each chain's first compacted row in cbase (-1:
  // none), and the next round's advance kernel sums that chain's chi^2
  // partials xpart[q xpstride + row], q < xnb, into its row likelihoods (and
  // adds the round's compacted rows to *xnet_rows); xpart null: rlogL is read.
  int* cbase;      // m entries
  const double* xpart;
  long xpstride;
  int xnb;
  unsigned long long* xnet_rows;
};

hipError_t launch_fill_int(int* p, long n, int v, hipStream_t s);
hipError_t launch_rounds_advance(int round, const RoundsParams& p, const Shape& sh, const DevBufs& b,
                                 const RoundBufs& r, hipStream_t s);
hipError_t launch_rows_from_points(long n, int d, const double* u, const RoundsParams& p,
                                   int state_f32, void* pts, float* xin, int* flag, hipStream_t s);
hipError_t launch_init_rows(int N, int d, uint64_t seed, const RoundsParams& p, int state_f32, void* u,
                            void* pts, float* xin, int* flag, hipStream_t s);
// A step's chains with a network likelihood in one persistent launch
// (k_emu_chains.hip): with split-bfloat16 layers the same results as the
// rounds driver, with FP32 layers (f32: the FP32 MFMA) the same to FP32
// rounding.  Eligible for FP32 state, P = 8 rows per chain and round, at most
// 8 layers, input width <= 32, hidden widths 256 or 512, output width 256,
// 512 or 1024, and the weights in the layout of the chosen arithmetic.
bool emu_chains_eligible(const NetDev& net, const RoundsParams& p, int state_f32, bool f32);
hipError_t launch_emu_chains(const RoundsParams& p, const NetDev& net, bool f32, const double* data,
                             const double* isig, const Shape& sh, const DevBufs& b, unsigned long long* net_rows,
                             hipStream_t s);
// W^T (N x K row major) into the FP32 MFMA block layout of N x Kp (Kp a
// multiple of 16, columns k >= K zero).
void fragq_layout_host(const float* wt, int N, int K, int Kp, float* out);
// analytic likelihood on rows (the batched driver with an analytic family)
hipError_t launch_rows_loglike(const Shape& sh, const LikDev& lik, long n, const void* pts,
                               const int* flag, double* out, const int* gate, hipStream_t s);

}  // namespace ns
