// Physics of eq. (3): the Euler system (B = 0, five variables) and ideal MHD
// in Gaussian units (eight variables), templated on the arithmetic type.
#pragma once
#include <hip/hip_runtime.h>

namespace ader {

// 1/x for the flux evaluations: correctly rounded in double; in float on the
// device the hardware reciprocal (within 1 ulp, one instruction where the
// IEEE divide takes about ten), an error far below what the FP32 bulk of the
// mixed path already carries.
__host__ __device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__host__ __device__ __forceinline__ float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// sqrt(x) for wave-speed estimates: correctly rounded in double; in float on
// the device the hardware square root (within 1 ulp).
__host__ __device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__host__ __device__ __forceinline__ float fsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}

template <class T>
struct Euler {
  static constexpr int NV = 5;

  // Physical flux along AXIS (0: F, 1: G, 2: H) of the conserved state u.
  template <int AXIS>
  __host__ __device__ static inline void flux(const T (&u)[5], T (&f)[5], T gam) {
    const T rinv = recip(u[0]);
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

  // Deviation form (mixed-precision path): the state at a point is carried as
  // du = u - ubar, ubar the zone average held in double, and the flux as
  // dF = F(ubar + du) - F(ubar).  Every term of dF below is a product with a
  // deviation, so its rounding error is relative to |dF| rather than |F|.
  struct Ref {
    T rho, m[3], v[3], h;   // density, momentum, velocity, E + p of ubar
  };
  __host__ __device__ static inline Ref make_ref(const double (&ub)[5], double gam) {
    const double ir = 1.0 / ub[0];
    const double v0 = ub[1] * ir, v1 = ub[2] * ir, v2 = ub[3] * ir;
    const double p = (gam - 1.0) * (ub[4] - 0.5 * (ub[1] * v0 + ub[2] * v1 + ub[3] * v2));
    Ref r;
    r.rho = T(ub[0]);
    r.m[0] = T(ub[1]); r.m[1] = T(ub[2]); r.m[2] = T(ub[3]);
    r.v[0] = T(v0); r.v[1] = T(v1); r.v[2] = T(v2);
    r.h = T(ub[4] + p);
    return r;
  }

  template <int AXIS>
  __host__ __device__ static inline void dflux(const Ref& r, const T (&du)[5], T (&f)[5], T gam) {
    const T rinv = recip(r.rho + du[0]);
    T dv[3], v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dv[a] = (du[1 + a] - r.v[a] * du[0]) * rinv;   // v - vbar
      v[a] = r.v[a] + dv[a];
    }
    // kinetic energy: m.v/2 - mbar.vbar/2 = (mbar.dv + dm.v)/2
    const T dk = T(0.5) * (r.m[0] * dv[0] + r.m[1] * dv[1] + r.m[2] * dv[2] +
                           du[1] * v[0] + du[2] * v[1] + du[3] * v[2]);
    const T dp = (gam - T(1)) * (du[4] - dk);
    f[0] = du[1 + AXIS];
#pragma unroll
    for (int a = 0; a < 3; ++a) f[1 + a] = du[1 + a] * v[AXIS] + r.m[a] * dv[AXIS];
    f[1 + AXIS] += dp;
    f[4] = (du[4] + dp) * v[AXIS] + r.h * dv[AXIS];
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
    const T rinv = recip(u[0]);
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

  // Deviation form, as for Euler: dF = F(ubar + du) - F(ubar).
  struct Ref {
    T rho, m[3], v[3], b[3], h, vb;   // ..., E + p + B^2/8pi, v.B of ubar
  };
  __host__ __device__ static inline Ref make_ref(const double (&ub)[8], double gam) {
    const double ir = 1.0 / ub[0];
    const double v0 = ub[1] * ir, v1 = ub[2] * ir, v2 = ub[3] * ir;
    const double pm = (ub[5] * ub[5] + ub[6] * ub[6] + ub[7] * ub[7]) * (1.0 / (8.0 * 3.14159265358979323846));
    const double p = (gam - 1.0) * (ub[4] - 0.5 * (ub[1] * v0 + ub[2] * v1 + ub[3] * v2) - pm);
    Ref r;
    r.rho = T(ub[0]);
    r.m[0] = T(ub[1]); r.m[1] = T(ub[2]); r.m[2] = T(ub[3]);
    r.v[0] = T(v0); r.v[1] = T(v1); r.v[2] = T(v2);
    r.b[0] = T(ub[5]); r.b[1] = T(ub[6]); r.b[2] = T(ub[7]);
    r.h = T(ub[4] + p + pm);
    r.vb = T(v0 * ub[5] + v1 * ub[6] + v2 * ub[7]);
    return r;
  }

  template <int AXIS>
  __host__ __device__ static inline void dflux(const Ref& r, const T (&du)[8], T (&f)[8], T gam) {
    constexpr T i4p = T(1.0 / (4.0 * 3.14159265358979323846));
    constexpr T i8p = T(1.0 / (8.0 * 3.14159265358979323846));
    const T rinv = recip(r.rho + du[0]);
    T dv[3], v[3], b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dv[a] = (du[1 + a] - r.v[a] * du[0]) * rinv;
      v[a] = r.v[a] + dv[a];
      b[a] = r.b[a] + du[5 + a];
    }
    const T dk = T(0.5) * (r.m[0] * dv[0] + r.m[1] * dv[1] + r.m[2] * dv[2] +
                           du[1] * v[0] + du[2] * v[1] + du[3] * v[2]);
    // magnetic pressure: (B.B - Bbar.Bbar)/8pi = dB.(Bbar + B)/8pi
    const T dpm = (du[5] * (r.b[0] + b[0]) + du[6] * (r.b[1] + b[1]) + du[7] * (r.b[2] + b[2])) * i8p;
    const T dpt = (gam - T(1)) * (du[4] - dk - dpm) + dpm;   // total pressure
    // v.B - vbar.Bbar = dv.B + vbar.dB
    const T dvb = dv[0] * b[0] + dv[1] * b[1] + dv[2] * b[2] +
                  r.v[0] * du[5] + r.v[1] * du[6] + r.v[2] * du[7];
    f[0] = du[1 + AXIS];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      f[1 + a] = du[1 + a] * v[AXIS] + r.m[a] * dv[AXIS] -
                 (du[5 + a] * b[AXIS] + r.b[a] * du[5 + AXIS]) * i4p;
    f[1 + AXIS] += dpt;
    f[4] = (du[4] + dpt) * v[AXIS] + r.h * dv[AXIS] -
           (du[5 + AXIS] * (r.vb + dvb) + r.b[AXIS] * dvb) * i4p;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      f[5 + a] = dv[AXIS] * b[a] + r.v[AXIS] * du[5 + a] - du[5 + AXIS] * v[a] - r.b[AXIS] * dv[a];
    f[5 + AXIS] = T(0);
  }
};

// Linearized dissipation of ideal MHD along AXIS (Sec. II.3): D = |A| du with
// |A| = R |Lambda| L of the seven-wave system -- primitive variables
// (rho, u_n, u_t1, u_t2, p, b_t1, b_t2), b = B / sqrt(4 pi), with b_n held at
// its frozen value -- at a frozen state, here the mean of the two barycentre
// primitive states.  Eigenvectors in the Roe & Balsara (1996) normalisation:
// with alpha_f^2 = (a^2 - c_s^2) / (c_f^2 - c_s^2), alpha_s^2 = (c_f^2 -
// a^2) / (c_f^2 - c_s^2), beta = b_t / |b_t| and s = sign(b_n), right vectors
// (sigma = -1, +1)
//   fast    (rho af, sig af cf, -sig as cs s beta, rho af a^2, as a sqrt(rho) beta)
//   Alfven  (0, 0, (-beta_2, beta_1), 0, sig s sqrt(rho) (beta_2, -beta_1))
//   slow    (rho as, sig as cs, sig af cf s beta, rho as a^2, -af a sqrt(rho) beta)
//   entropy (1, 0, 0, 0, 0, 0, 0)
// and the dual left vectors; beta = (1, 1)/sqrt(2) when b_t = 0, and
// (alpha_f, alpha_s) = (1, 0) when c_f = c_s.  Conserved jumps are mapped to
// primitive ones and back with the Jacobian of the variable change at the
// frozen state; the normal-field row of D is zero.
template <class T, int AXIS>
struct MhdEigen {
  static constexpr int T1 = AXIS == 0 ? 1 : 0, T2 = AXIS == 2 ? 1 : 2;
  T rho, sr, un, u1, u2, q2, bn, b1, b2, a2, a, cf, cs, ca, af, as, be1, be2, sg, gm1;

  __host__ __device__ MhdEigen(const T (&ul)[8], const T (&ur)[8], T gam) {
    constexpr T i4p = T(1.0 / (4.0 * 3.14159265358979323846));
    const T isq4p = sqrt(i4p);
    const T il = T(1) / ul[0], ir = T(1) / ur[0];
    rho = T(0.5) * (ul[0] + ur[0]);
    T v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = T(0.5) * (ul[1 + d] * il + ur[1 + d] * ir);
    const T p = T(0.5) * (Mhd<T>::pressure(ul, gam) + Mhd<T>::pressure(ur, gam));
    T B[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) B[d] = T(0.5) * (ul[5 + d] + ur[5 + d]);
    un = v[AXIS];
    u1 = v[T1];
    u2 = v[T2];
    q2 = un * un + u1 * u1 + u2 * u2;
    bn = B[AXIS] * isq4p;
    b1 = B[T1] * isq4p;
    b2 = B[T2] * isq4p;
    gm1 = gam - T(1);
    sr = sqrt(rho);
    a2 = gam * p / rho;
    a = sqrt(a2);
    const T ca2 = bn * bn / rho;
    const T bt2 = (b1 * b1 + b2 * b2) / rho;
    const T s = a2 + ca2 + bt2;
    const T disc = s * s - T(4) * a2 * ca2;
    const T cf2 = T(0.5) * (s + sqrt(disc > T(0) ? disc : T(0)));
    const T cs2 = cf2 > T(0) ? a2 * ca2 / cf2 : T(0);    // c_f^2 c_s^2 = a^2 c_a^2
    cf = sqrt(cf2);
    cs = sqrt(cs2);
    ca = sqrt(ca2);
    const T bperp = sqrt(b1 * b1 + b2 * b2);
    if (bperp > T(0)) {
      be1 = b1 / bperp;
      be2 = b2 / bperp;
    } else {
      be1 = be2 = T(0.70710678118654752);
    }
    const T dd = cf2 - cs2;
    if (dd > T(0)) {
      const T f = (a2 - cs2) / dd, g = (cf2 - a2) / dd;
      af = sqrt(fmin(fmax(f, T(0)), T(1)));
      as = sqrt(fmin(fmax(g, T(0)), T(1)));
    } else {
      af = T(1);
      as = T(0);
    }
    sg = bn >= T(0) ? T(1) : T(-1);
  }

  __host__ __device__ void apply(const T (&du)[8], T (&D)[8]) const {
    constexpr T s4p = T(3.5449077018110321);   // sqrt(4 pi)
    // conserved -> primitive jump at the frozen state
    const T dr = du[0];
    const T irho = T(1) / rho;
    const T dun = (du[1 + AXIS] - un * dr) * irho;
    const T du1 = (du[1 + T1] - u1 * dr) * irho;
    const T du2 = (du[1 + T2] - u2 * dr) * irho;
    const T db1 = du[5 + T1] / s4p, db2 = du[5 + T2] / s4p;
    const T dp = gm1 * (du[4] - (un * du[1 + AXIS] + u1 * du[1 + T1] + u2 * du[1 + T2]) +
                        T(0.5) * q2 * dr - (b1 * db1 + b2 * db2));
    // wave strengths (left vectors) times |lambda|
    const T ia2 = T(0.5) / a2;
    const T isr = T(1) / sr;
    const T par = dp * irho;                                  // common parts
    const T bdu = be1 * du1 + be2 * du2;                      // beta . du_t
    const T bdb = (be1 * db1 + be2 * db2) * isr;              // beta . db_t / sqrt(rho)
    const T xdu = -be2 * du1 + be1 * du2;                     // beta^perp . du_t
    const T xdb = (-be2 * db1 + be1 * db2) * isr;
    T w[7];
    {
      const T fa = af * par + as * a * bdb, fb = af * cf * dun - as * cs * sg * bdu;
      w[0] = fabs(un - cf) * ia2 * (fa - fb);   // fast -
      w[1] = fabs(un + cf) * ia2 * (fa + fb);   // fast +
      const T sa = as * par - af * a * bdb, sb = as * cs * dun + af * cf * sg * bdu;
      w[2] = fabs(un - cs) * ia2 * (sa - sb);   // slow -
      w[3] = fabs(un + cs) * ia2 * (sa + sb);   // slow +
      w[4] = fabs(un - ca) * T(0.5) * (xdu + sg * xdb);   // Alfven -
      w[5] = fabs(un + ca) * T(0.5) * (xdu - sg * xdb);   // Alfven +
      w[6] = fabs(un) * (dr - dp / a2);                    // entropy
    }
    // primitive result: sum of w_k R_k
    const T fsum = w[0] + w[1], fdif = w[1] - w[0];
    const T ssum = w[2] + w[3], sdif = w[3] - w[2];
    const T asum = w[4] + w[5], adif = w[5] - w[4];
    const T r_ = rho * (af * fsum + as * ssum) + w[6];
    const T un_ = af * cf * fdif + as * cs * sdif;
    const T tpar = -as * cs * sg * fdif + af * cf * sg * sdif;   // along beta
    const T u1_ = tpar * be1 - be2 * asum;
    const T u2_ = tpar * be2 + be1 * asum;
    const T p_ = rho * a2 * (af * fsum + as * ssum);
    const T bpar = a * sr * (as * fsum - af * ssum);
    const T b1_ = bpar * be1 + sg * sr * be2 * adif;
    const T b2_ = bpar * be2 - sg * sr * be1 * adif;
    // primitive -> conserved
    D[0] = r_;
    D[1 + AXIS] = rho * un_ + un * r_;
    D[1 + T1] = rho * u1_ + u1 * r_;
    D[1 + T2] = rho * u2_ + u2 * r_;
    D[4] = T(0.5) * q2 * r_ + rho * (un * un_ + u1 * u1_ + u2 * u2_) + p_ / gm1 + b1 * b1_ + b2 * b2_;
    D[5 + AXIS] = T(0);
    D[5 + T1] = s4p * b1_;
    D[5 + T2] = s4p * b2_;
  }
};

// Flux evaluators for the generated per-zone code.  PointFlux takes the state
// at a point and returns its physical flux; DeviationFlux takes the deviation
// of the state from the zone average and returns the deviation of the flux
// (exact algebra, the mixed-precision path).  kDeviation tells the generated
// code whether point values carry the zone average; comp(c) is the slot of
// variable c in the arrays it is handed.
template <class P, class T>
struct PointFlux {
  static constexpr bool kDeviation = false;
  static constexpr int comp(int c) { return c; }
  T gam;
  template <int AXIS, int NV>
  __host__ __device__ inline void flux(const T (&u)[NV], T (&f)[NV]) const {
    P::template flux<AXIS>(u, f, gam);
  }
};

template <class P, class T>
struct DeviationFlux {
  static constexpr bool kDeviation = true;
  static constexpr int comp(int c) { return c; }
  typename P::Ref ref;
  T gam;
  template <int AXIS, int NV>
  __host__ __device__ inline void flux(const T (&du)[NV], T (&f)[NV]) const {
    P::template dflux<AXIS>(ref, du, f, gam);
  }
};

}  // namespace ader
