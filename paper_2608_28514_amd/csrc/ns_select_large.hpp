// ns_select_large.hpp -- launcher of the worst-m selection at scale
// (k_select_large.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ns {

// workspace bytes of launch_select_large (device, 256-byte aligned)
size_t select_large_work_bytes();
// out[0..m-1] = indices of the m smallest (order key of logL, index), ascending;
// passes (may be null): number of streaming passes made over logL
hipError_t launch_select_large(const double* logL, long N, int m, int* out, void* work, int* passes,
                               hipStream_t s);

}  // namespace ns
