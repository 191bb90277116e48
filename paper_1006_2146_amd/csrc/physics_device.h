// Physics of eq. (3): the Euler system (B = 0, five variables) and ideal MHD
// in Gaussian units (eight variables), templated on the arithmetic type.
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

  template <int AXIS>
  __host__ __device__ static inline T fast_speed(const T (&u)[5], T gam) {
    return sqrt(gam * pressure(u, gam) / u[0]);
  }
};

template <class T>
struct Mhd {
  static constexpr int NV = 8;

  // Physical flux along AXIS of u = (rho, m, E, B): momentum and energy
  // fluxes carry the magnetic pressure B^2/8pi and stresses B_i B_j/4pi; the
  // induction part is v_AXIS B - B_AXIS v (zero in the AXIS component).
  template <int AXIS>
  __host__ __device__ static inline void flux(const T (&u)[8], T (&f)[8], T gam) {
    const T rinv = T(1) / u[0];
    const T vx = u[1] * rinv, vy = u[2] * rinv, vz = u[3] * rinv;
    const T bx = u[5], by = u[6], bz = u[7];
    const T b2 = bx * bx + by * by + bz * bz;
    const T pmag = b2 * T(1.0 / (8.0 * 3.14159265358979323846));
    const T p = (gam - T(1)) * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz) - pmag);
    const T pt = p + pmag;
    const T v[3] = {vx, vy, vz};
    const T b[3] = {bx, by, bz};
    const T vn = v[AXIS];
    const T bn4 = b[AXIS] * T(1.0 / (4.0 * 3.14159265358979323846));
    const T vb = vx * bx + vy * by + vz * bz;
    f[0] = u[1 + AXIS];
    f[1] = u[1] * vn - bx * bn4;
    f[2] = u[2] * vn - by * bn4;
    f[3] = u[3] * vn - bz * bn4;
    f[1 + AXIS] += pt;
    f[4] = (u[4] + pt) * vn - bn4 * vb;
    f[5] = vn * bx - b[AXIS] * vx;
    f[6] = vn * by - b[AXIS] * vy;
    f[7] = vn * bz - b[AXIS] * vz;
    f[5 + AXIS] = T(0);
  }

  __host__ __device__ static inline T pressure(const T (&u)[8], T gam) {
    const T b2 = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    return (gam - T(1)) * (u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0] -
                           b2 * T(1.0 / (8.0 * 3.14159265358979323846)));
  }

  // fast magnetosonic speed along AXIS
  template <int AXIS>
  __host__ __device__ static inline T fast_speed(const T (&u)[8], T gam) {
    const T rho = u[0];
    const T a2 = gam * pressure(u, gam) / rho;
    const T inv4pr = T(1) / (T(4.0 * 3.14159265358979323846) * rho);
    const T b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * inv4pr;
    const T bn2 = u[5 + AXIS] * u[5 + AXIS] * inv4pr;
    const T s = a2 + b2;
    const T disc = s * s - T(4) * a2 * bn2;
    return sqrt(T(0.5) * (s + sqrt(disc > T(0) ? disc : T(0))));
  }
};

}  // namespace ader
