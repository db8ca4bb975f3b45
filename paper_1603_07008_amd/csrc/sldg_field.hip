// Self-consistent field of a 1D-1V (x, v) problem for the v-sweep of the
// split step (L. Einkemmer, arXiv 1603.07008, section II: the Vlasov equation
// with the field E(x); the field equation is Gauss's law of the normalised
// Vlasov-Poisson system, dE/dx = rho - mean(rho), E periodic with zero mean,
// rho(x) = int f dv).
//
// The density in x cell i is the Legendre expansion r_j(i) = h_v sum_iv
// c(i, iv; mode (j, 0)) (a v cell integrates P_jv to h_v for jv = 0 and to 0
// otherwise).  E is the zero-mean antiderivative of rho - mean(rho), a
// polynomial of degree k+1 per cell; the v-sweep displaces the line through
// x cell i by E(x_i) dt / h_v (each line uses its transverse cell centre).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sldg_field.h"

namespace sldg {

template <class T>
__device__ __forceinline__ double as_double(T v) {
  if constexpr (sizeof(T) == 2) return (double)(float)v;
  else return (double)v;
}

// Partial v-sums of the (j, 0) modes: workgroup (x, j, z) sums v rows
// [z * rows, (z+1) * rows) of x cells [256x, 256x+256) of mode j.
template <class T>
__global__ __launch_bounds__(256) void density_partial_kernel(FieldPlanes fp, int32_t nx,
                                                              int32_t nv, int32_t rows,
                                                              double* __restrict__ part) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  const int32_t j = (int32_t)blockIdx.y, z = (int32_t)blockIdx.z;
  if (i >= nx) return;
  const int32_t v0 = z * rows, v1 = min(nv, v0 + rows);
  double acc = 0.0;
  if (fp.lo[j]) {
    const double* p = static_cast<const double*>(fp.plane[j]);
    for (int32_t iv = v0; iv < v1; ++iv) acc += p[(int64_t)iv * nx + i];
  } else {
    const T* p = static_cast<const T*>(fp.plane[j]);
    for (int32_t iv = v0; iv < v1; ++iv) acc += as_double(p[(int64_t)iv * nx + i]);
  }
  part[((int64_t)z * gridDim.y + j) * nx + i] = acc;
}

constexpr int kFieldThreads = 256;

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kFieldThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One workgroup: the density moments, the mean density, the face values of
// the antiderivative (a serial scan along x), its cell means, the zero-mean
// constant, and E and the displacement at the cell centres.  `half[j]` is
// int_{-1}^{0} P_j.
__global__ __launch_bounds__(kFieldThreads) void field_solve_kernel(
    const double* __restrict__ part, int32_t nz, int32_t o, int32_t nx, double hx, double hv,
    double dt, double h0, double h1, double h2, double h3, double* __restrict__ r,
    double* __restrict__ faces, double* __restrict__ shift_out, double* __restrict__ field_out) {
  __shared__ double sh[kFieldThreads];
  const double half[4] = {h0, h1, h2, h3};
  // density moments r[j][i] = h_v * sum over the v chunks
  for (int32_t i = threadIdx.x; i < nx; i += kFieldThreads)
    for (int32_t j = 0; j < o; ++j) {
      double acc = 0.0;
      for (int32_t z = 0; z < nz; ++z) acc += part[((int64_t)z * o + j) * nx + i];
      r[(int64_t)j * nx + i] = hv * acc;
    }
  __syncthreads();
  double loc = 0.0;
  for (int32_t i = threadIdx.x; i < nx; i += kFieldThreads) loc += r[i];
  const double rbar = block_sum(loc, sh) / nx;
  // face values of the antiderivative of rho - rbar, from 0 at the left end
  if (threadIdx.x == 0) {
    double f = 0.0;
    faces[0] = 0.0;
    for (int32_t i = 0; i < nx; ++i) {
      f += hx * (r[i] - rbar);
      faces[i + 1] = f;
    }
  }
  __syncthreads();
  // cell means: F_i + h/2 (r0 - rbar) - h/6 r1; the constant making the mean 0
  loc = 0.0;
  for (int32_t i = threadIdx.x; i < nx; i += kFieldThreads)
    loc += faces[i] + 0.5 * hx * (r[i] - rbar) - (o > 1 ? hx / 6.0 * r[(int64_t)nx + i] : 0.0);
  const double C = -block_sum(loc, sh) / nx;
  for (int32_t i = threadIdx.x; i < nx; i += kFieldThreads) {
    double g = (r[i] - rbar) * half[0];
    for (int32_t j = 1; j < o; ++j) g += r[(int64_t)j * nx + i] * half[j];
    const double E = faces[i] + C + 0.5 * hx * g;
    shift_out[i] = E * dt / hv;
    if (field_out) field_out[i] = E;
  }
}

template <class T>
static hipError_t launch_field_t(const FieldPlanes& fp, int o, int32_t nx, int32_t nv,
                                 double hx, double hv, double dt, double* scratch,
                                 double* shift_out, double* field_out, hipStream_t st) {
  const int32_t nz = field_chunks(nv);
  const int32_t rows = (nv + nz - 1) / nz;
  double* part = scratch;                                  // [nz][o][nx]
  double* r = part + (int64_t)nz * o * nx;                 // [o][nx]
  double* faces = r + (int64_t)o * nx;                     // [nx + 1]
  dim3 grid((unsigned)((nx + 255) / 256), (unsigned)o, (unsigned)nz);
  density_partial_kernel<T><<<grid, 256, 0, st>>>(fp, nx, nv, rows, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // int_{-1}^{0} P_j for j = 0..3
  field_solve_kernel<<<1, kFieldThreads, 0, st>>>(part, nz, o, nx, hx, hv, dt, 1.0, -0.5, 0.0,
                                                  0.125, r, faces, shift_out, field_out);
  return hipGetLastError();
}

int32_t field_chunks(int32_t nv) { return nv < 32 ? (nv > 0 ? nv : 1) : 32; }

int64_t field_scratch_doubles(int o, int32_t nx, int32_t nv) {
  return (int64_t)field_chunks(nv) * o * nx + (int64_t)o * nx + nx + 1;
}

hipError_t launch_field(int tier, const FieldPlanes& fp, int o, int32_t nx, int32_t nv,
                        double hx, double hv, double dt, double* scratch, double* shift_out,
                        double* field_out, hipStream_t st) {
  switch (tier) {
    case 0: return launch_field_t<double>(fp, o, nx, nv, hx, hv, dt, scratch, shift_out, field_out, st);
    case 1: return launch_field_t<float>(fp, o, nx, nv, hx, hv, dt, scratch, shift_out, field_out, st);
    case 2: return launch_field_t<__bf16>(fp, o, nx, nv, hx, hv, dt, scratch, shift_out, field_out, st);
    case 3: return launch_field_t<_Float16>(fp, o, nx, nv, hx, hv, dt, scratch, shift_out, field_out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sldg
