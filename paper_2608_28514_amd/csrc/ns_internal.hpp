// ns_internal.hpp -- host-side view of the device buffers of one sampler
// context and the kernel launchers that operate on them.
#pragma once
#include <hip/hip_runtime.h>
#include "ns_device.hpp"

namespace ns {

// Device pointers of one context.  Sizes: N live points, d dims, M = max batch
// (chains), T = history capacity, nodes = 2^(D+1)-1.
struct DevBufs {
  void* u;              // N x d, state precision
  double* logL;         // N
  int* label;           // N (cluster node)
  int* order;           // N (ascending (logL, slot))
  int* seeds;           // M
  int* seeds2;          // M: seeds of the next step, written by the end-of-step kernel
  double* tau;          // M (shrink thresholds)
  double* tau2;         // M (next step)
  double* LW;           // M (logL of the m worst, ascending)
  double* LW2;          // M (next step)
  void* new_u;          // M x d
  double* new_logL;     // M
  int* chain_stat;      // M x kStatW: evals, oob, stepout caps, shrink caps, screened
  double* hist_logL;    // T x M (row t, column chain)
  void* hist_u;         // M x T x d
  int* hist_n;          // M
  void* draws;          // M x n_iter x (d + kDrawExtra): per-iteration draw blocks of the slice kernel
  // cluster tree
  int* nodeof;          // N: deepest tree node of each point
  int* count;           // nodes
  int* accepted;        // nodes
  int* split_ok;        // nodes
  double* logV;         // nodes
  double* logV_eff;     // nodes
  double* centre;       // nodes x 32
  double* cov;          // nodes x 32 x 32
  double* chol;         // nodes x 32 x 32
  float* chol_f;        // nodes x 32 x 32
  // the root by the multi-workgroup split (cluster_root_split); null otherwise
  void* root_work;      // split workspace (cluster_split_work_bytes)
  double* root_stats;   // mean (32), covariance (d x d, stride d; 32 x 32 room), centres (2 x 32),
                        // then the children's counts, means and covariances (kRootChild ..)
  unsigned char* root_side;  // N: side of each point at the root split
  // dead store
  double* dead_u;       // cap x d
  double* dead_logL;    // cap
  RunState* st;
  HostProgress* prog;   // device view of the host progress word (may be null)
};

constexpr int kStatW = 8;  // ints per chain in chain_stat
// Draw block of one slice iteration of the fused slice kernel: d direction
// entries, the bracket offset a0 and kShrinkPre shrink uniforms.
constexpr int kShrinkPre = 32;
constexpr int kDrawExtra = 1 + kShrinkPre;

struct Shape {
  int N, d, T, nodes, depth;
  int state_f32;   // sampler state in FP32 (else FP64)
  int lik_f32;     // analytic likelihood in FP32 (else FP64)
};

struct SliceParams {
  int m;
  int n_iter;
  double w;
  int max_stepout;
  int max_shrink;
  int corr;
  uint64_t seed;
};

// kernels.  Every launcher enqueues on `s` and returns hipGetLastError().
hipError_t launch_init_points(const Shape& sh, const DevBufs& b, const LikDev& lik, uint64_t seed,
                              hipStream_t s);
hipError_t launch_loglike_points(const Shape& sh, const LikDev& lik, const double* u, long n,
                                 double* out, hipStream_t s);
hipError_t launch_select(const Shape& sh, const DevBufs& b, int m, int corr, uint64_t seed,
                         hipStream_t s);
hipError_t launch_select_order(const double* logL, int N, int* order, hipStream_t s);
// The fused slice kernel reads the draw blocks that launch_slice_draws writes
// (call it first, on the same stream).
hipError_t launch_slice_draws(const Shape& sh, const DevBufs& b, const SliceParams& p, hipStream_t s);
hipError_t launch_slice(const Shape& sh, const DevBufs& b, const LikDev& lik, const SliceParams& p,
                        hipStream_t s);
// sel_m > 0: also select the next step's m worst points and seeds into
// seeds2 / tau2 / LW2 (and order); ignored unless correct_selects_next(sh).
hipError_t launch_correct(const Shape& sh, const DevBufs& b, int m, int corr, int K,
                          double stop_frac, int sel_m, uint64_t seed, hipStream_t s);
bool correct_selects_next(const Shape& sh);
hipError_t launch_correct_arrays(int m, int corr, int K, int T, const double* wlogL,
                                 const double* nlogL, const double* P, const double* hist,
                                 const int* hist_n, int* acc_code, int* acc_hslot, double* acc_logL,
                                 int* rej_code, int* rej_hslot, double* rej_logL, hipStream_t s);
// wait_limit: polls of a grid barrier before it gives up (0: the default)
hipError_t launch_cluster(const Shape& sh, const DevBufs& b, double p, int nmin, int iters,
                          double eps, int wait_limit, hipStream_t s);
// True when the root of the tree is computed by the multi-workgroup split
// (FP32 state, a split below the root, and more points than one workgroup
// holds in LDS); the context then provides root_work, root_stats, root_side.
bool cluster_root_split(const Shape& sh);
constexpr int kRootChild = 32 + 32 * 32 + 2 * 32;
constexpr int kRootStats = kRootChild + 2 + 2 * 32 + 2 * 32 * 32;
// Regularise every node with at least two points (the tree as a whole).
hipError_t launch_regularise_all(const Shape& sh, const DevBufs& b, int nmin, double eps, hipStream_t s);
hipError_t launch_final_logZ(const Shape& sh, const DevBufs& b, double* out3, hipStream_t s);
hipError_t launch_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, long n,
                         uint32_t* out, hipStream_t s);

}  // namespace ns
