// HIP kernels of one ADER-CG step on a periodic mesh (gfx950): one thread per
// zone over the per-zone operations of zone_ops.h, plus the wavefront/block
// reductions of the CFL time step.
#pragma once
#include <hip/hip_runtime.h>

#include "zone_ops.h"

namespace ader {

// The FP32 (mixed-precision) kernels run the deviation form, the FP64 ones
// the point form.
template <class T>
constexpr bool kDeviation = sizeof(T) == 4;

template <class T, int M, int AXIS, int NVAR>
__global__ void __launch_bounds__(256) k_weno_sweep(const double* __restrict__ U,
                                                    T* __restrict__ W, Grid g) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) weno_sweep_zone<T, M, AXIS, NVAR>(U, W, g, n);
}

template <class T, int NVAR>
__global__ void __launch_bounds__(256) k_minmod(const double* __restrict__ U,
                                                T* __restrict__ W, Grid g) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) minmod_zone<T, NVAR>(U, W, g, n);
}

template <class T, int M>
__global__ void __launch_bounds__(256) k_bface(const double* __restrict__ B, double* __restrict__ B0,
                                               T* __restrict__ BN, Grid g) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) bface_zone<T, M>(B, B0, BN, g, n);
}

template <class T, int ORDER, int FORM>
__global__ void __launch_bounds__(128) k_predict_mhd(const double* __restrict__ U,
                                                     const T* __restrict__ W,
                                                     const double* __restrict__ B0,
                                                     const T* __restrict__ WB,
                                                     const T* __restrict__ BN, T* __restrict__ PK,
                                                     Grid g, const double* __restrict__ dt,
                                                     double inv_dx, double inv_dy, double inv_dz,
                                                     double gam) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N)
    predict_zone_mhd<T, ORDER, FORM, kDeviation<T>>(U, W, B0, WB, BN, PK, g, *dt, inv_dx, inv_dy,
                                                    inv_dz, gam, n);
}

template <class T>
__global__ void __launch_bounds__(256) k_face_flux_mhd(const double* __restrict__ U,
                                                       const double* __restrict__ B0,
                                                       const T* __restrict__ PK,
                                                       double* __restrict__ F,
                                                       double* __restrict__ FE, Grid g, double gam) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) face_flux_zone_mhd<T, kDeviation<T>>(U, B0, PK, F, FE, g, gam, n);
}

__global__ void __launch_bounds__(256) k_edge_e(const double* __restrict__ FE,
                                                double* __restrict__ E, Grid g) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) edge_e_zone(FE, E, g, n);
}

// eq. (6) for the hydro variables and eq. (8) for the face fields
__global__ void __launch_bounds__(256) k_update_mhd(double* __restrict__ U, double* __restrict__ B,
                                                    const double* __restrict__ F,
                                                    const double* __restrict__ E, Grid g,
                                                    const double* __restrict__ dt, double dx,
                                                    double dy, double dz) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) {
    const double h = *dt;
    update_zone(U, F, g, h, dx, dy, dz, n);
    ct_zone(B, E, g, h, dx, dy, dz, n);
  }
}

template <class T, int ORDER, int FORM>
__global__ void __launch_bounds__(128) k_predict(const double* __restrict__ U,
                                                 const T* __restrict__ W,
                                                 T* __restrict__ PK, Grid g,
                                                 const double* __restrict__ dt,
                                                 double inv_dx, double inv_dy,
                                                 double inv_dz, double gam) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N)
    predict_zone<T, ORDER, FORM, kDeviation<T>>(U, W, PK, g, *dt, inv_dx, inv_dy, inv_dz, gam, n);
}

template <class T, int RS>
__global__ void __launch_bounds__(256) k_face_flux(const double* __restrict__ U,
                                                   const T* __restrict__ PK,
                                                   double* __restrict__ F, Grid g, double gam) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) face_flux_zone<T, RS, kDeviation<T>>(U, PK, F, g, gam, n);
}

__global__ void __launch_bounds__(256) k_update(double* __restrict__ U, const double* __restrict__ F,
                                                Grid g, const double* __restrict__ dt,
                                                double dx, double dy, double dz) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < g.N) update_zone(U, F, g, *dt, dx, dy, dz, n);
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// B == nullptr: Euler; otherwise MHD with the face fields B
__global__ void __launch_bounds__(256) k_dt_partial(const double* __restrict__ U,
                                                    const double* __restrict__ B, Grid g, double gam,
                                                    double dx, double dy, double dz,
                                                    double* __restrict__ partial,
                                                    int* __restrict__ bad) {
  __shared__ double red[4];
  __shared__ int redbad[4];
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double rate = 0.0;
  int isbad = 0;
  if (n < g.N)
    rate = B ? dt_rate_zone_mhd(U, B, g, gam, dx, dy, dz, n, isbad)
             : dt_rate_zone(U, g, gam, dx, dy, dz, n, isbad);
  rate = wave_max(rate);
  int wb = isbad;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) wb |= __shfl_xor(wb, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = rate;
    redbad[wid] = wb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    int b = redbad[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      r = fmax(r, red[q]);
      b |= redbad[q];
    }
    partial[blockIdx.x] = r;
    bad[blockIdx.x] = b;
  }
}

__global__ void __launch_bounds__(1024) k_dt_final(const double* __restrict__ partial,
                                                   const int* __restrict__ bad, int nparts,
                                                   double cfl, double* __restrict__ dt,
                                                   int* __restrict__ status) {
  __shared__ double red[16];
  __shared__ int redbad[16];
  double r = 0.0;
  int b = 0;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) {
    r = fmax(r, partial[q]);
    b |= bad[q];
  }
  r = wave_max(r);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) b |= __shfl_xor(b, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = r;
    redbad[wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      r = fmax(r, red[q]);
      b |= redbad[q];
    }
    r = fmax(r, red[0]);
    b |= redbad[0];
    if (b || !(r > 0.0)) {
      *status = 1;
    } else {
      *dt = cfl / r;
    }
  }
}

__global__ void k_set_scalar(double* __restrict__ p, double value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = value;
}
}  // namespace ader
