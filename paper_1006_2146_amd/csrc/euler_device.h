// Device-side Euler physics of eq. (3) with B = 0: fluxes, primitives and
// signal speeds, templated on the arithmetic type.
#pragma once
#include <hip/hip_runtime.h>

namespace ader {

template <class T>
struct Euler {
  static constexpr int NV = 5;

  // Physical flux along AXIS (0: F, 1: G, 2: H) of the conserved state u.
  template <int AXIS>
  __host__ __device__ static inline void flux(const T (&u)[5], T (&f)[5], T gam) {
    const T rinv = T(1) / u[0];
    const T vn = u[1 + AXIS] * rinv;
    const T ke = T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * rinv;
    const T p = (gam - T(1)) * (u[4] - ke);
    f[0] = u[1 + AXIS];
    f[1] = u[1] * vn;
    f[2] = u[2] * vn;
    f[3] = u[3] * vn;
    f[1 + AXIS] += p;
    f[4] = (u[4] + p) * vn;
  }

  __host__ __device__ static inline T pressure(const T (&u)[5], T gam) {
    return (gam - T(1)) * (u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
  }
};

}  // namespace ader
