// ns_cluster_large.hpp -- launcher of one cluster-tree node's statistics and
// k-means split for large point sets (k_cluster_large.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ns {

size_t cluster_split_work_bytes();
// u: N x d FP32 (row major); mean: d; cov: d x d (stride d); centres: 2 x 32
// (row 0 first centre, row 1 second); side: N bytes; passes (may be null):
// streaming passes made over u
hipError_t launch_cluster_split(const float* u, long N, int d, int iters, double* mean, double* cov,
                                double* centres, unsigned char* side, void* work, int* passes, hipStream_t s);
// The same quantities in one cooperative launch (mean, farthest points,
// Lloyd passes; the covariance pass after it) for 16 < d <= 32 and at most 64
// tiles of 256 points; hipErrorNotSupported otherwise (use the above).
// cstats (may be null): the two sides' statistics as children of the node:
// counts [0..2), means [2 + 32 c ..), unbiased covariances [66 + 1024 c ..)
// (d x d, stride d).  A grid barrier polls at most wait_limit times (0: 2^24);
// if it gives up, the launch sets *fault (may be null) and its outputs are
// not valid.
hipError_t launch_cluster_split_coop(const float* u, long N, int d, int iters, double* mean, double* cov,
                                     double* centres, unsigned char* side, double* cstats, void* work,
                                     int* fault, int wait_limit, hipStream_t s);

}  // namespace ns
