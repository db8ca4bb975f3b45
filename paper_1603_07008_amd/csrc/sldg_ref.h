// Reference-bandwidth kernels beside the sweeps (sldg_ref.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sldg {

// nplanes planes of n16 16-byte words; each thread copies one word offset of
// T consecutive planes in turn.
hipError_t launch_plane_copy16(const void* src, void* dst, int64_t n16, int32_t nplanes,
                               int32_t T, hipStream_t st);

}  // namespace sldg
