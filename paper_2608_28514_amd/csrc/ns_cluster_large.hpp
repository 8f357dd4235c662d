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

}  // namespace ns
