// Self-consistent field of 1D-1V problems (sldg_field.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sldg {

// Planes of the modes (j, 0), j = 0..k, of an (x, v) state: plane[j] points
// at N_x * N_v values, FP64 when lo[j], else in the tier's storage type.
struct FieldPlanes {
  const void* plane[4];
  int32_t lo[4];
};

// v chunks of the partial density sums, and the doubles of scratch a field
// solve needs.
int32_t field_chunks(int32_t nv);
int64_t field_scratch_doubles(int o, int32_t nx, int32_t nv);

// shift_out[i] = E(x_i) dt / h_v, field_out[i] = E(x_i) (optional).
hipError_t launch_field(int tier, const FieldPlanes& fp, int o, int32_t nx, int32_t nv,
                        double hx, double hv, double dt, double* scratch, double* shift_out,
                        double* field_out, hipStream_t st);

}  // namespace sldg
