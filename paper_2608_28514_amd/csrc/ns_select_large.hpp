// ns_select_large.hpp -- launcher of the worst-m selection at scale
// (k_select_large.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ns {

// workspace bytes of launch_select_large (device, 256-byte aligned)
size_t select_large_work_bytes();
// device address of the static selection workspace of the current device
// (select_large_work_bytes() bytes, 256-byte aligned), resolved on first use
hipError_t select_large_static_work(void** out);
// out[0..m-1] = indices of the m smallest (order key of logL, index), ascending;
// passes (may be null): number of streaming passes made over logL
hipError_t launch_select_large(const double* logL, long N, int m, int* out, void* work, int* passes,
                               hipStream_t s);

}  // namespace ns
