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
#include <math.h>
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

constexpr int kFieldThreads = 1024;

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
// the antiderivative (a block-wide scan along x), its cell means, the
// zero-mean constant, and E and the displacement at the cell centres.
// `half[j]` is int_{-1}^{0} P_j.
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
  // face values of the antiderivative of rho - rbar, from 0 at the left end:
  // each thread sums a contiguous chunk of cells, an inclusive scan of the
  // chunk sums (fixed order) gives each chunk's starting face, and the thread
  // writes its chunk's faces
  const int32_t per = (nx + kFieldThreads - 1) / kFieldThreads;
  const int32_t i0 = min(nx, (int32_t)threadIdx.x * per), i1 = min(nx, i0 + per);
  double chunk = 0.0;
  for (int32_t i = i0; i < i1; ++i) chunk += hx * (r[i] - rbar);
  sh[threadIdx.x] = chunk;
  __syncthreads();
  for (int off = 1; off < kFieldThreads; off <<= 1) {
    const double v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  double f = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;   // sum of the chunks before
  __syncthreads();
  if (threadIdx.x == 0) faces[0] = 0.0;
  for (int32_t i = i0; i < i1; ++i) {
    f += hx * (r[i] - rbar);
    faces[i + 1] = f;
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

int32_t field_chunks(int32_t nv) { return nv < 8 ? (nv > 0 ? nv : 1) : 8; }

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

// ---------------------------------------------------------------------------
// 2D-2V problems (x1, x2, v1, v2).  Gauss's law div E = rho - mean(rho) with a
// curl-free periodic E = -grad phi, solved spectrally on the x-cell means of
// rho (h_v1 h_v2 times the sum over the v cells of the cell mean c_0): the
// DFT of the cell means is divided by the Fourier symbol of cell averaging,
// sinc(kappa_1 h_1/2) sinc(kappa_2 h_2/2), and E_hat = -i kappa rho_hat /
// |kappa|^2 (mean and Nyquist modes dropped); E at the x cell centres.  The
// transforms are direct DFTs (N1, N2 <= kMaxDft) with twiddles from a table
// in LDS and exact integer phase reduction; all arithmetic in FP64.
// ---------------------------------------------------------------------------

// Partial sums over v cells [z rows, (z+1) rows) of the mode-0 plane for x
// cells [256 blockIdx.x, +256).
template <class T>
__global__ __launch_bounds__(256) void density2_partial_kernel(const void* plane, int64_t nxx,
                                                               int64_t nslab, int64_t rows,
                                                               double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t z = blockIdx.y;
  if (i >= nxx) return;
  const int64_t s0 = z * rows, s1 = s0 + rows < nslab ? s0 + rows : nslab;
  const T* p = static_cast<const T*>(plane);
  double acc = 0.0;
  for (int64_t s = s0; s < s1; ++s) acc += as_double(p[s * nxx + i]);
  part[z * nxx + i] = acc;
}

__global__ __launch_bounds__(256) void density2_final_kernel(const double* __restrict__ part,
                                                             int32_t nz, int64_t nxx,
                                                             double hvv, double* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nxx) return;
  double acc = 0.0;
  for (int32_t z = 0; z < nz; ++z) acc += part[(int64_t)z * nxx + i];
  rho[i] = hvv * acc;
}

// tw[r] = exp(2 pi i r / n), r < n, filled by the workgroup.
__device__ __forceinline__ void fill_twiddles(double2* tw, int32_t n) {
  for (int32_t r = threadIdx.x; r < n; r += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * r / n, &sn, &cs);
    tw[r] = make_double2(cs, sn);
  }
  __syncthreads();
}

// Forward DFT along x1 of the real cell means: thread t = k1 + N1 i2,
// C[t] = sum_i1 rho[i1 + N1 i2] exp(-2 pi i k1 i1 / N1).
__global__ __launch_bounds__(256) void dft_x1_kernel(const double* __restrict__ rho, int32_t n1,
                                                     int32_t n2, double2* __restrict__ C) {
  extern __shared__ double2 tw[];
  fill_twiddles(tw, n1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n1 * n2) return;
  const int32_t k1 = (int32_t)(t % n1), i2 = (int32_t)(t / n1);
  const double* row = rho + (int64_t)i2 * n1;
  double re = 0.0, im = 0.0;
  int32_t r = 0;
  for (int32_t i1 = 0; i1 < n1; ++i1) {
    const double v = row[i1];
    re = fma(v, tw[r].x, re);
    im = fma(-v, tw[r].y, im);
    r += k1;
    if (r >= n1) r -= n1;
  }
  C[t] = make_double2(re, im);
}

// Wave number 2 pi m / (n h), m the index taken in (-n/2, n/2]; nyq when m is
// the Nyquist index of an even n.
__device__ __forceinline__ double wave_number(int32_t j, int32_t n, double h, bool* nyq) {
  const int32_t m = j <= n / 2 ? j : j - n;
  *nyq = (n % 2 == 0) && (j == n / 2);
  return 2.0 * M_PI * m / (n * h);
}

// sin(pi m / n) / (pi m / n), the cell-average symbol at index j.
__device__ __forceinline__ double cell_sinc(int32_t j, int32_t n) {
  const int32_t m = j <= n / 2 ? j : j - n;
  if (m == 0) return 1.0;
  const double z = (double)m / n;
  return sinpi(z) / (M_PI * z);
}

// Forward DFT along x2 and the field symbol: thread t = k1 + N1 k2,
// R = sum_i2 C[k1 + N1 i2] exp(-2 pi i k2 i2 / N2), then
// E_hat_f = -i kappa_f (R / sincs) / |kappa|^2.
__global__ __launch_bounds__(256) void dft_x2_solve_kernel(const double2* __restrict__ C,
                                                           int32_t n1, int32_t n2, double h1,
                                                           double h2, double2* __restrict__ E1h,
                                                           double2* __restrict__ E2h) {
  extern __shared__ double2 tw[];
  fill_twiddles(tw, n2);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n1 * n2) return;
  const int32_t k1 = (int32_t)(t % n1), k2 = (int32_t)(t / n1);
  double re = 0.0, im = 0.0;
  int32_t r = 0;
  for (int32_t i2 = 0; i2 < n2; ++i2) {
    const double2 c = C[k1 + (int64_t)n1 * i2];
    const double2 w = tw[r];                       // exp(+...); the forward uses its conjugate
    re = fma(c.x, w.x, fma(c.y, w.y, re));
    im = fma(c.y, w.x, fma(-c.x, w.y, im));
    r += k2;
    if (r >= n2) r -= n2;
  }
  bool ny1, ny2;
  const double q1 = wave_number(k1, n1, h1, &ny1), q2 = wave_number(k2, n2, h2, &ny2);
  double2 e1 = make_double2(0.0, 0.0), e2 = e1;
  if (!ny1 && !ny2 && (k1 != 0 || k2 != 0)) {
    const double sc = cell_sinc(k1, n1) * cell_sinc(k2, n2);
    const double pre = re / sc, pim = im / sc;
    const double kk = q1 * q1 + q2 * q2;
    // -i kappa (pre + i pim) = kappa pim - i kappa pre
    e1 = make_double2(q1 * pim / kk, -q1 * pre / kk);
    e2 = make_double2(q2 * pim / kk, -q2 * pre / kk);
  }
  E1h[t] = e1;
  E2h[t] = e2;
}

// Inverse DFT along x2 of both fields: thread t = k1 + N1 i2,
// D_f[t] = sum_k2 E_hat_f[k1 + N1 k2] exp(2 pi i k2 i2 / N2).
__global__ __launch_bounds__(256) void idft_x2_kernel(const double2* __restrict__ E1h,
                                                      const double2* __restrict__ E2h, int32_t n1,
                                                      int32_t n2, double2* __restrict__ D1,
                                                      double2* __restrict__ D2) {
  extern __shared__ double2 tw[];
  fill_twiddles(tw, n2);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n1 * n2) return;
  const int32_t k1 = (int32_t)(t % n1), i2 = (int32_t)(t / n1);
  double a_re = 0.0, a_im = 0.0, b_re = 0.0, b_im = 0.0;
  int32_t r = 0;
  for (int32_t k2 = 0; k2 < n2; ++k2) {
    const double2 w = tw[r];
    const double2 a = E1h[k1 + (int64_t)n1 * k2], b = E2h[k1 + (int64_t)n1 * k2];
    a_re = fma(a.x, w.x, fma(-a.y, w.y, a_re));
    a_im = fma(a.x, w.y, fma(a.y, w.x, a_im));
    b_re = fma(b.x, w.x, fma(-b.y, w.y, b_re));
    b_im = fma(b.x, w.y, fma(b.y, w.x, b_im));
    r += i2;
    if (r >= n2) r -= n2;
  }
  D1[t] = make_double2(a_re, a_im);
  D2[t] = make_double2(b_re, b_im);
}

// Inverse DFT along x1, real part, 1 / (N1 N2): thread t = i1 + N1 i2.
__global__ __launch_bounds__(256) void idft_x1_kernel(const double2* __restrict__ D1,
                                                      const double2* __restrict__ D2, int32_t n1,
                                                      int32_t n2, double dt, double hv1,
                                                      double hv2, double* __restrict__ shift1,
                                                      double* __restrict__ shift2,
                                                      double* __restrict__ field) {
  extern __shared__ double2 tw[];
  fill_twiddles(tw, n1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nxx = (int64_t)n1 * n2;
  if (t >= nxx) return;
  const int32_t i1 = (int32_t)(t % n1), i2 = (int32_t)(t / n1);
  const double2* d1 = D1 + (int64_t)i2 * n1;
  const double2* d2 = D2 + (int64_t)i2 * n1;
  double e1 = 0.0, e2 = 0.0;
  int32_t r = 0;
  for (int32_t k1 = 0; k1 < n1; ++k1) {
    const double2 w = tw[r];
    e1 = fma(d1[k1].x, w.x, fma(-d1[k1].y, w.y, e1));
    e2 = fma(d2[k1].x, w.x, fma(-d2[k1].y, w.y, e2));
    r += i1;
    if (r >= n1) r -= n1;
  }
  const double inv = 1.0 / (double)nxx;
  e1 *= inv;
  e2 *= inv;
  shift1[t] = e1 * dt / hv1;
  shift2[t] = e2 * dt / hv2;
  if (field) {
    field[t] = e1;
    field[nxx + t] = e2;
  }
}

int32_t field2_chunks(int64_t nxx, int64_t nslab) {
  int64_t nz = nslab < 256 ? nslab : 256;
  const int64_t cap = ((int64_t)1 << 22) / (nxx > 0 ? nxx : 1);
  if (nz > cap) nz = cap;
  return (int32_t)(nz > 0 ? nz : 1);
}

int64_t field2_scratch_doubles(int32_t n1, int32_t n2, int64_t nslab) {
  const int64_t nxx = (int64_t)n1 * n2;
  return (int64_t)field2_chunks(nxx, nslab) * nxx + 11 * nxx + 1;   // + 1: double2 alignment
}

template <class T>
static hipError_t launch_density2(const Field2Args& a, int32_t nz, int64_t nxx, double* part,
                                  hipStream_t st) {
  const int64_t rows = (a.nslab + nz - 1) / nz;
  dim3 grid((unsigned)((nxx + 255) / 256), (unsigned)nz);
  density2_partial_kernel<T><<<grid, 256, 0, st>>>(a.plane0, nxx, a.nslab, rows, part);
  return hipGetLastError();
}

hipError_t launch_field2(int tier, const Field2Args& a, double* scratch, hipStream_t st) {
  const int64_t nxx = (int64_t)a.n1 * a.n2;
  if (a.n1 < 1 || a.n2 < 1 || a.n1 > kMaxDft || a.n2 > kMaxDft) return hipErrorInvalidValue;
  const int32_t nz = field2_chunks(nxx, a.nslab);
  double* part = scratch;                               // [nz][nxx]
  double* rho = part + (int64_t)nz * nxx;                // [nxx]
  const int64_t cofs = ((int64_t)nz * nxx + nxx + 1) & ~(int64_t)1;   // 16-byte aligned
  double2* C = reinterpret_cast<double2*>(scratch + cofs);  // [nxx] complex
  double2* E1h = C + nxx;
  double2* E2h = E1h + nxx;
  double2* D1 = E2h + nxx;
  double2* D2 = D1 + nxx;
  hipError_t e;
  if (a.lo0) e = launch_density2<double>(a, nz, nxx, part, st);
  else {
    switch (tier) {
      case 0: e = launch_density2<double>(a, nz, nxx, part, st); break;
      case 1: e = launch_density2<float>(a, nz, nxx, part, st); break;
      case 2: e = launch_density2<__bf16>(a, nz, nxx, part, st); break;
      case 3: e = launch_density2<_Float16>(a, nz, nxx, part, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)((nxx + 255) / 256);
  density2_final_kernel<<<g, 256, 0, st>>>(part, nz, nxx, a.hv1 * a.hv2, rho);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds1 = sizeof(double2) * a.n1, lds2 = sizeof(double2) * a.n2;
  dft_x1_kernel<<<g, 256, lds1, st>>>(rho, a.n1, a.n2, C);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dft_x2_solve_kernel<<<g, 256, lds2, st>>>(C, a.n1, a.n2, a.h1, a.h2, E1h, E2h);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  idft_x2_kernel<<<g, 256, lds2, st>>>(E1h, E2h, a.n1, a.n2, D1, D2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  idft_x1_kernel<<<g, 256, lds1, st>>>(D1, D2, a.n1, a.n2, a.dt, a.hv1, a.hv2, a.shift1,
                                       a.shift2, a.field);
  return hipGetLastError();
}

}  // namespace sldg
