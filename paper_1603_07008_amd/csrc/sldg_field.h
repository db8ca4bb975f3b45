// Self-consistent fields of 1D-1V and 2D-2V problems (sldg_field.hip).
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

// 2D-2V: the cell-mean plane (mode 0) of an (x1, x2, v1, v2) state, the
// grid and cell widths, and the outputs (each N1 * N2, x1 fastest).
struct Field2Args {
  const void* plane0;      // N1 N2 N_v1 N_v2 values
  int32_t lo0;             // plane0 is FP64 (else the tier's storage type)
  int32_t n1, n2;          // x cells
  int64_t nslab;           // v cells, N_v1 N_v2
  double h1, h2, hv1, hv2, dt;
  double* shift1;          // E_1 dt / h_v1
  double* shift2;          // E_2 dt / h_v2
  double* field;           // optional: E_1 then E_2
};

constexpr int32_t kMaxDft = 2048;   // largest N1, N2 (the twiddle table is in LDS)

int32_t field2_chunks(int64_t nxx, int64_t nslab);
int64_t field2_scratch_doubles(int32_t n1, int32_t n2, int64_t nslab);

hipError_t launch_field2(int tier, const Field2Args& a, double* scratch, hipStream_t st);

}  // namespace sldg
