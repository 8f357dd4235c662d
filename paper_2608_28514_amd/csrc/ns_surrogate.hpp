// ns_surrogate.hpp -- counters and launchers of the learned pre-screen
// (k_surrogate.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "ns_device.hpp"

namespace ns {

constexpr uint32_t kStreamSurrogate = 4;
constexpr int kNormLen = 2 + 2 * kMaxD;   // [mu, s, input means (32), input 1/std (32)]

// Device-side counters of the batched network likelihood.
struct SurrCounters {
  unsigned long long pairs;          // (theta, logL) pairs appended to the replay ring
  unsigned long long emu_rows;       // rows evaluated by the true likelihood network
  unsigned long long screened_seen;  // rows the surrogate placed below threshold - margin
  unsigned long long audited;        // screened rows evaluated anyway
  unsigned long long false_screens;  // audited rows that cleared their threshold
};

// chunk_cnt: 2 ints per chunk of 256 rows (scratch shared by the two passes).
// xf (may be null): the compacted inputs also as three fragment-major
// bfloat16 planes (hi, mid, lo) of 32 columns, plane stride xfplane; columns
// d..31 are not written.
hipError_t launch_screen(int M, int d, int screening, double margin, int audit_period, const int* flag,
                         const double* rthr, const float* yhat, const float* norm, const float* xin,
                         int* sflag, int* idx, int* aud, float* xc, __bf16* xf, long xfplane, int* count,
                         double* rlogL, SurrCounters* sc, int* chunk_cnt, const int* gate, hipStream_t s);
// M: rows of the round (upper bound of count[0]).  The logL of compacted row
// i is clogL[i], or, with part non-null, -1/2 sum_q part[q M + i] over the nb
// chi^2 column blocks of emu_forward_logL.
hipError_t launch_scatter(int M, int d, const int* count, const int* idx, const int* aud, const double* clogL,
                          const double* part, int nb, const double* rthr, const float* xc, double* rlogL,
                          float* rep_x, double* rep_y, long cap, SurrCounters* sc, const int* gate,
                          hipStream_t s);
hipError_t launch_sample_batch(int B, int d, uint64_t seed, uint32_t call, uint32_t iter, const float* rep_x,
                               const double* rep_y, long cap, const SurrCounters* sc, const double* LW,
                               const RunState* st, const double* root_centre, const double* root_cov,
                               const double* lo_box, const double* span_box, double floor_below, float* Xb,
                               float* yb, float* norm, hipStream_t s);
hipError_t launch_standardize(long n, int d, const float* x, const float* norm, float* xs, const int* gate,
                              hipStream_t s);
hipError_t launch_mse_grad(int B, const float* yhat, const float* y, float* dY, float* loss, hipStream_t s);
hipError_t launch_adam(long n, float lr, float b1, float b2, float eps, int t, float* p, const float* g,
                       float* m, float* v, hipStream_t s);
hipError_t launch_norm_apply(long n, const float* norm, float* y, hipStream_t s);
hipError_t launch_glorot(long n, int fan_in, int fan_out, uint64_t seed, uint32_t layer, float* w, hipStream_t s);

}  // namespace ns
