// Reference-bandwidth kernels of libsldg beside the plain copy: the access
// pattern of the projection sweeps (L. Einkemmer, arXiv 1603.07008, section
// II-A: one load and one store per coefficient) without their arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sldg_ref.h"

namespace sldg {

// Plane copy (reference bandwidth of the sweeps' access pattern): nplanes
// planes of n16 16-byte words; workgroup (x, y) copies words [256x, 256x+256)
// of planes [yT, yT+T), one plane after the other, as a sweep thread walks the
// planes of its run of spectator tuples.
__global__ __launch_bounds__(256) void plane_copy16_kernel(const uint4* __restrict__ src,
                                                           uint4* __restrict__ dst, int64_t n16,
                                                           int32_t nplanes, int32_t T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n16) return;
  const int32_t p0 = (int32_t)blockIdx.y * T, p1 = min(nplanes, p0 + T);
  for (int32_t p = p0; p < p1; ++p) dst[(int64_t)p * n16 + i] = src[(int64_t)p * n16 + i];
}

hipError_t launch_plane_copy16(const void* src, void* dst, int64_t n16, int32_t nplanes,
                               int32_t T, hipStream_t st) {
  if (n16 <= 0 || nplanes <= 0) return hipSuccess;
  const int64_t bx = (n16 + 255) / 256, by = (nplanes + T - 1) / T;
  if (bx > 0x7fffffff || by > 65535) return hipErrorInvalidValue;
  plane_copy16_kernel<<<dim3((unsigned)bx, (unsigned)by), 256, 0, st>>>(
      static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16, nplanes, T);
  return hipGetLastError();
}

}  // namespace sldg
