// Per-zone operations of one ADER-CG step on a periodic mesh, callable from
// the gfx950 kernels (ader_kernels.h) and, for CPU tests of the kernel logic,
// from a host build.
//
// Data in HBM, all structure-of-arrays with the zone index n = (k ny + j) nx + i
// fastest, so consecutive lanes of a wavefront touch consecutive addresses:
//   U   double [5][N]            conserved zone averages (eq. 6 state)
//   W   T      [LS-1][5][N]      reconstructed spatial modes w_2..w_LS (eq. 10-12)
//   PK  T      [6][3][5][N]      face-side packets: per side (x-, x+, y-, y+,
//                                z-, z+) the barycentre state (eq. 54), the
//                                face average of u (eq. 55) and of the normal
//                                flux (App. D)
//   F   double [3][5][N]         numerical flux at the lower x/y/z face of each
//                                zone (eq. 56 or the linearized flux)
// T is double on the FP64 path and float on the mixed path; U, F, the update
// and dt stay double on both.  The mixed path runs in deviation form (DEV):
// the FP32 quantities are differences from the zone average (states) or from
// the flux of the zone average (fluxes), which is held in double, so FP32
// rounding is relative to the small variation inside a zone and not to the
// state itself; the face flux adds the FP64 flux of the two zone averages.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "physics_device.h"
#include "generated/ader_scheme.h"

namespace ader {

// One zone's walk down the rows of an SoA array (row stride N): the address
// advances by one row per access.  On the device an empty asm fences each
// step, so the compiler keeps it as one 64-bit add instead of hoisting a
// separate row offset per row out of the zone loop, which it cannot hold in
// scalar registers and spills.
template <class P>
__host__ __device__ __forceinline__ P* next_row(P* p, long long N) {
#if defined(__HIP_DEVICE_COMPILE__)
  // fenced as a global-memory pointer, so accesses through it stay global
  __attribute__((address_space(1))) P* g = (__attribute__((address_space(1))) P*)p;
  g += N;
  asm("" : "+v"(g));
  return (P*)g;
#else
  return p + N;
#endif
}

// Cursor over one zone's rows of an SoA array: row(r) moves the address by
// r - (current row) rows with next_row and returns the element, so accesses
// in increasing row order cost one add each.
template <class P>
struct RowCursor {
  P* p;
  long long N;
  int at;
  __host__ __device__ RowCursor(P* base, long long stride, long long n, int row0 = 0)
      : p(base + (long long)row0 * stride + n), N(stride), at(row0) {}
  __host__ __device__ __forceinline__ P& row(int r) {
    if (r != at) {
      p = next_row(p, (long long)(r - at) * N);
      at = r;
    }
    return *p;
  }
};

// One periodic mesh inside the arrays: nx*ny*nz = N zones stored at indices
// base .. base+N-1 of arrays whose per-variable stride is S (S = N and base =
// 0 for a lone problem; a batch concatenates its problems).
struct Grid {
  int nx, ny, nz;
  long long N;
  long long S;
  long long base;
};

__host__ __device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__host__ __device__ __forceinline__ long long zone_of(int i, int j, int k, const Grid& g) {
  return g.base + ((long long)k * g.ny + j) * g.nx + i;
}

// (i, j, k) of the array index n of a zone of g
__host__ __device__ __forceinline__ void zone_ijk(const Grid& g, long long n, int& i, int& j, int& k) {
  const long long l = n - g.base;
  const long long row = l / g.nx;
  i = (int)(l - row * g.nx);
  k = (int)(row / g.ny);
  j = (int)(row - (long long)k * g.ny);
}

// Position of spatial mode P_a(xi) P_b(eta) P_c(zeta) in the order of
// eq. (10)-(12) (0-based).
__host__ __device__ constexpr int spatial_mode(int a, int b, int c) {
  return (a == 0 && b == 0 && c == 0) ? 0
       : (a == 1 && b == 0 && c == 0) ? 1
       : (a == 0 && b == 1 && c == 0) ? 2
       : (a == 0 && b == 0 && c == 1) ? 3
       : (a == 2 && b == 0 && c == 0) ? 4
       : (a == 0 && b == 2 && c == 0) ? 5
       : (a == 0 && b == 0 && c == 2) ? 6
       : (a == 1 && b == 1 && c == 0) ? 7
       : (a == 0 && b == 1 && c == 1) ? 8
       : (a == 1 && b == 0 && c == 1) ? 9
       : (a == 3 && b == 0 && c == 0) ? 10
       : (a == 0 && b == 3 && c == 0) ? 11
       : (a == 0 && b == 0 && c == 3) ? 12
       : (a == 2 && b == 1 && c == 0) ? 13
       : (a == 2 && b == 0 && c == 1) ? 14
       : (a == 1 && b == 2 && c == 0) ? 15
       : (a == 0 && b == 2 && c == 1) ? 16
       : (a == 1 && b == 0 && c == 2) ? 17
       : (a == 0 && b == 1 && c == 2) ? 18
       : (a == 1 && b == 1 && c == 1) ? 19
       : -1;
}

template <int M>
struct Ls { static constexpr int value = M == 2 ? 4 : M == 3 ? 10 : 20; };

// ---------------------------------------------------------------------------
// Centred WENO in one direction (the reading of Sec. II.1 used throughout:
// all M-zone stencils covering the zone, smoothness indicator of the form of
// eq. (24)/(29), weights lambda/(eps+IS)^2 with lambda 100 for the central
// (order 3) or the two inner (order 4) stencils and 1 otherwise).
// d[0..2M-2] are the averages at offsets -(M-1)..(M-1); m[1..M-1] receive the
// moments of P_1..P_{M-1}.
// ---------------------------------------------------------------------------
template <class T, int M>
__host__ __device__ __forceinline__ void weno1d(const T (&d)[2 * M - 1], T (&m)[M]) {
  constexpr double kEps = 1.0e-12;
  if constexpr (M == 3) {
    T c0[3], c1[3], c2[3];
    ader_gen::Weno3<T>::cand0(d, c0);
    ader_gen::Weno3<T>::cand1(d, c1);
    ader_gen::Weno3<T>::cand2(d, c2);
    const T is0 = c0[1] * c0[1] + T(13.0 / 3.0) * c0[2] * c0[2];
    const T is1 = c1[1] * c1[1] + T(13.0 / 3.0) * c1[2] * c1[2];
    const T is2 = c2[1] * c2[1] + T(13.0 / 3.0) * c2[2] * c2[2];
    const T e0 = T(kEps) + is0, e1 = T(kEps) + is1, e2 = T(kEps) + is2;
    const T q0 = e0 * e0, q1 = e1 * e1, q2 = e2 * e2;
    T a0, a1, a2, inv;
    if constexpr (sizeof(T) == 4) {
      // FP32: lambda_s / q_s with hardware reciprocals (1 ulp each)
      a0 = recip(q0);
      a1 = T(100) * recip(q1);
      a2 = recip(q2);
      inv = recip(a0 + a1 + a2);
    } else {
      // FP64: the same weights times q0 q1 q2 (no division), one division
      // for the normalisation
      a0 = q1 * q2;
      a1 = T(100) * (q0 * q2);
      a2 = q0 * q1;
      inv = T(1) / (a0 + a1 + a2);
    }
    m[1] = (a0 * c0[1] + a1 * c1[1] + a2 * c2[1]) * inv;
    m[2] = (a0 * c0[2] + a1 * c1[2] + a2 * c2[2]) * inv;
  } else {
    T c[4][4];
    ader_gen::Weno4<T>::cand0(d, c[0]);
    ader_gen::Weno4<T>::cand1(d, c[1]);
    ader_gen::Weno4<T>::cand2(d, c[2]);
    ader_gen::Weno4<T>::cand3(d, c[3]);
    T qq[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T t = c[s][1] + T(0.1) * c[s][3];
      const T is = t * t + T(13.0 / 3.0) * c[s][2] * c[s][2] + T(781.0 / 20.0) * c[s][3] * c[s][3];
      const T e = T(kEps) + is;
      qq[s] = e * e;
    }
    T a[4], inv;
    if constexpr (sizeof(T) == 4) {
      // FP32: lambda_s / q_s with hardware reciprocals (1 ulp each)
#pragma unroll
      for (int s = 0; s < 4; ++s) a[s] = ((s == 1 || s == 2) ? T(100) : T(1)) * recip(qq[s]);
      inv = recip(a[0] + a[1] + a[2] + a[3]);
    } else {
      // FP64: the same weights times q0 q1 q2 q3 (no division), one division
      // for the normalisation
      const T p01 = qq[0] * qq[1], p23 = qq[2] * qq[3];
      a[0] = qq[1] * p23;
      a[1] = T(100) * (qq[0] * p23);
      a[2] = T(100) * (p01 * qq[3]);
      a[3] = p01 * qq[2];
      inv = T(1) / (a[0] + a[1] + a[2] + a[3]);
    }
#pragma unroll
    for (int q = 1; q < 4; ++q)
      m[q] = (a[0] * c[0][q] + a[1] * c[1][q] + a[2] * c[2][q] + a[3] * c[3][q]) * inv;
  }
}

// One sweep of the dimension-by-dimension reconstruction along AXIS.
// x: the zone averages give the x-moments (a,0,0);  y: each field (a,0,0),
// a <= M-2, gives (a,b,0);  z: each field (a,b,0), a+b <= M-2, gives (a,b,c);
// moments of total degree > M-1 are not formed.
// NVAR fields; their zone averages (mode 0) are the double array U[NVAR][N]
// (the conserved variables, or for MHD the zone field b_0) and their modes
// 2..L_S go to W[L_S-1][NVAR][N].
template <class T, int M, int AXIS, int NVAR = 5>
__host__ __device__ __forceinline__ void weno_sweep_zone(const double* __restrict__ U,
                                                         T* __restrict__ W, const Grid& g,
                                                         long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  constexpr int R = M - 1;
  long long idx[2 * R + 1];
#pragma unroll
  for (int o = -R; o <= R; ++o) {
    if constexpr (AXIS == 0) idx[o + R] = zone_of(wrap(i + o, g.nx), j, k, g);
    if constexpr (AXIS == 1) idx[o + R] = zone_of(i, wrap(j + o, g.ny), k, g);
    if constexpr (AXIS == 2) idx[o + R] = zone_of(i, j, wrap(k + o, g.nz), g);
  }
#pragma unroll
  for (int a = 0; a <= M - 1; ++a) {
#pragma unroll
    for (int b = 0; b <= M - 1; ++b) {
      // source field of this sweep and how many new moments it yields
      int nout;
      if constexpr (AXIS == 0) nout = (a == 0 && b == 0) ? M - 1 : 0;
      else if constexpr (AXIS == 1) nout = (b == 0 && a <= M - 2) ? M - 1 - a : 0;
      else nout = (a + b <= M - 2) ? M - 1 - a - b : 0;
      if (nout == 0) continue;
      const int src = spatial_mode(a, b, 0);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        // the zone averages enter as differences to the centre zone, formed
        // in double (the moments do not see a constant shift)
        T d[2 * M - 1];
#pragma unroll
        for (int q = 0; q < 2 * R + 1; ++q)
          d[q] = src == 0 ? T(U[(long long)v * g.S + idx[q]] - U[(long long)v * g.S + n])
                          : W[((long long)(src - 1) * NVAR + v) * g.S + idx[q]];
        T mo[M];
        weno1d<T, M>(d, mo);
#pragma unroll
        for (int c = 1; c <= M - 1; ++c) {
          if (c > nout) continue;
          int dst;
          if constexpr (AXIS == 0) dst = spatial_mode(c, 0, 0);
          else if constexpr (AXIS == 1) dst = spatial_mode(a, c, 0);
          else dst = spatial_mode(a, b, c);
          W[((long long)(dst - 1) * NVAR + v) * g.S + n] = mo[c];
        }
      }
    }
  }
}

// Second order: per axis the minmod of the two one-sided differences
// (the limiter of the second-order workload).
template <class T, int NVAR = 5>
__host__ __device__ __forceinline__ void minmod_zone(const double* __restrict__ U,
                                                     T* __restrict__ W, const Grid& g,
                                                     long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long nb[3][2] = {
      {zone_of(wrap(i - 1, g.nx), j, k, g), zone_of(wrap(i + 1, g.nx), j, k, g)},
      {zone_of(i, wrap(j - 1, g.ny), k, g), zone_of(i, wrap(j + 1, g.ny), k, g)},
      {zone_of(i, j, wrap(k - 1, g.nz), g), zone_of(i, j, wrap(k + 1, g.nz), g)}};
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    const double c = U[(long long)v * g.S + n];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double fwd = U[(long long)v * g.S + nb[ax][1]] - c;
      const double bwd = c - U[(long long)v * g.S + nb[ax][0]];
      double s = 0.0;
      if (fwd * bwd > 0.0) s = fabs(fwd) < fabs(bwd) ? fwd : bwd;
      W[((long long)ax * NVAR + v) * g.S + n] = T(s);
    }
  }
}

// ---------------------------------------------------------------------------
// Positivity.  The paper's scheme has no positivity treatment: in the check
// mode (the default) a zone whose polynomial has rho <= 0 or P <= 0 at a
// check point flags its problem (the step then reports an unphysical
// state) and nothing is changed.  The limit mode is an opt-in safeguard:
// one Zhang-Shu scaling factor per zone polynomial, computed in double.
// NV = 5 (Euler) or 8 (MHD: the pressure carries B^2/8pi).
// ---------------------------------------------------------------------------

// Positivity handling of a kernel launch: the mode and, per problem, the
// violation flag (check mode) and the count of scaled zone polynomials
// (limit mode).  at(p) points the two at problem p.
struct PosCtl {
  int limit;
  int* bad;
  unsigned int* limited;
  int sink;   // offset of the sink slots (outcomes that must not count)
  __host__ __device__ PosCtl at(int p) const { return PosCtl{limit, bad + p, limited + p, 0}; }
  __host__ __device__ PosCtl sunk(int p) const {
    return PosCtl{limit, bad + sink + p, limited + sink + p, 0};
  }
};

// Outcome of the exact pass of a zone: true if its modes are to be scaled by
// theta (limit mode, theta < 1, counted); a violation of the check mode
// (theta < 0) flags the problem and scales nothing.
__host__ __device__ inline bool pos_scales(const PosCtl& pc, double theta) {
  if (!(theta < 1.0)) return false;
  if (theta < 0.0) {
    *pc.bad = 1;
    return false;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  atomicAdd(pc.limited, 1u);
#else
  ++*pc.limited;
#endif
  return true;
}
template <int NV>
__host__ __device__ __forceinline__ double pressure_of(const double (&u)[NV], double gam) {
  double e = u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
  if constexpr (NV == 8) e -= (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * (1.0 / (8.0 * 3.14159265358979323846));
  return (gam - 1.0) * e;
}

// limit: the scaling factor theta; else the check (violation set when a
// point has rho <= 0 or P <= 0) and result() is -1 on a violation, 1 if not.
template <class T, int NV>
struct PosTheta {
  double ub[NV];
  double eps_rho, eps_p, gam, theta;
  bool limit, violation;

  __host__ __device__ PosTheta(const double (&w0)[NV], double g, bool lim)
      : gam(g), theta(1.0), limit(lim), violation(false) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] = w0[v];
    eps_rho = 1.0e-8 * ub[0];
    eps_p = 1.0e-8 * pressure_of<NV>(ub, gam);
  }

  // Euler: smallest t in (0, 1] where the pressure along ub + t du falls to
  // eps_p: root of rho(t)(E(t) - e) - |m(t)|^2/2 = a t^2 + b t + c
  __host__ __device__ double pressure_root(const double (&du)[NV]) const {
    const double e = eps_p / (gam - 1.0);
    const double a = du[0] * du[4] - 0.5 * (du[1] * du[1] + du[2] * du[2] + du[3] * du[3]);
    const double b = ub[0] * du[4] + du[0] * (ub[4] - e) - (ub[1] * du[1] + ub[2] * du[2] + ub[3] * du[3]);
    const double c = ub[0] * (ub[4] - e) - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]);
    double t;
    if (a == 0.0) {
      t = -c / b;
    } else {
      const double disc = sqrt(fmax(b * b - 4.0 * a * c, 0.0));
      const double qq = -0.5 * (b + (b >= 0.0 ? disc : -disc));
      double t1 = qq / a, t2 = c / qq;
      if (!(__builtin_isfinite(t1) && t1 >= 0.0)) t1 = 2.0;
      if (!(__builtin_isfinite(t2) && t2 >= 0.0)) t2 = 2.0;
      t = fmin(t1, t2);
    }
    return fmin(fmax(t, 0.0), 1.0);
  }

  // MHD: the pressure is concave along the line where rho > 0; its bound is
  // located by bisection, keeping the admissible end
  __host__ __device__ double pressure_bisect(const double (&du)[NV]) const {
    double lo = 0.0, hi = 1.0;
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
      const double mid = 0.5 * (lo + hi);
      double v[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = ub[q] + mid * du[q];
      const bool ok = v[0] > 0.0 && pressure_of<NV>(v, gam) >= eps_p;
      if (ok) lo = mid; else hi = mid;
    }
    return lo;
  }

  // theta = min over points of the largest admissible scale along the line
  // from the zone average to the point: the density bound (linear) and the
  // first crossing of the pressure bound; the same value as scaling for
  // density first and then for pressure.
  __host__ __device__ double result() const { return limit ? theta : (violation ? -1.0 : 1.0); }

  __host__ __device__ void operator()(const double (&u)[NV]) {
    const double p = pressure_of<NV>(u, gam);
    if (!limit) {
      if (!(u[0] > 0.0) || !(p > 0.0)) violation = true;
      return;
    }
    if (u[0] < eps_rho || p < eps_p) {
      double t = 1.0;
      if (u[0] < eps_rho) t = (ub[0] - eps_rho) / (ub[0] - u[0]);
      double du[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) du[v] = u[v] - ub[v];
      if constexpr (NV == 5) t = fmin(t, pressure_root(du));
      else t = fmin(t, pressure_bisect(du));
      theta = fmin(theta, t);
    }
  }
};

// Cheap scan of the same points: flags a zone whose polynomial comes near
// the bounds (within a factor 2 of the bounds, plus a margin of 64 rounding
// units of T for the error of the point values, so that rounding in T never
// hides a violation); only such zones run the exact pass in double.  In the
// deviation form the point values come without the zone average, which the
// scan adds back.
template <class T, int NV, bool DEV>
struct PosScan {
  static constexpr bool kDeviation = DEV;
  static constexpr T kSlack = T(64) * T(sizeof(T) == 4 ? 5.96e-8 : 1.11e-16);
  T base[NV];
  T eps_rho, eps_e;
  int near = 0;
  __host__ __device__ static T rho_internal(const T (&u)[NV]) {
    // rho times the internal energy per volume, free of divisions
    T r = u[0] * u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]);
    if constexpr (NV == 8)
      r -= u[0] * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * T(1.0 / (8.0 * 3.14159265358979323846));
    return r;
  }
  __host__ __device__ PosScan(const double (&w0)[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) base[v] = DEV ? T(w0[v]) : T(0);
    T u0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u0[v] = T(w0[v]);
    eps_rho = (T(2.0e-8) + kSlack) * u0[0];
    eps_e = T(2.0e-8) * rho_internal(u0) / u0[0];
  }
  // rho >= eps_rho and rho (internal energy) >= rho eps_e, with the margin
  __host__ __device__ void operator()(const T (&du)[NV]) {
    T u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = DEV ? base[v] + du[v] : du[v];
    const int ok = int(u[0] >= eps_rho) &
                   int(rho_internal(u) >= u[0] * eps_e + kSlack * fabs(u[0] * u[4]));
    near |= ok ^ 1;
  }
};

// Exact pass for a flagged zone: a runtime loop over the check points with
// the basis values from the scheme's tables, so the rare path stays small;
// the scaling factor (limit) or the check's result (see PosTheta).
// The zone average w0 comes in double; the modes w[1..] (and e) are summed in
// double, so both forms (w[0] is not read) give the same point values.
template <int NP, int LS, class T, int NV>
__host__ __device__ double theta_spatial_tab(const double (&w0)[NV], const T (&w)[LS][NV],
                                             const double (&phi)[NP][LS], double gam, bool limit) {
  PosTheta<T, NV> acc(w0, gam, limit);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = w0[v];
#pragma unroll
      for (int m = 1; m < LS; ++m) s += phi[p][m] * double(w[m][v]);
      u[v] = s;
    }
    acc(u);
  }
  return acc.result();
}

template <int NP, int LS, int NE, class T, int NV>
__host__ __device__ double theta_facial_tab(const double (&w0)[NV], const T (&w)[LS][NV],
                                            const T (&e)[NE][NV],
                                            const double (&phi)[NP][LS + NE], double gam,
                                            bool limit) {
  PosTheta<T, NV> acc(w0, gam, limit);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = w0[v];
#pragma unroll
      for (int m = 1; m < LS; ++m) s += phi[p][m] * double(w[m][v]);
#pragma unroll
      for (int m = 0; m < NE; ++m) s += phi[p][LS + m] * double(e[m][v]);
      u[v] = s;
    }
    acc(u);
  }
  return acc.result();
}

// The flux evaluator of each form.
template <class P, class T, bool DEV>
struct FluxOf;
template <class P, class T>
struct FluxOf<P, T, false> {
  using type = PointFlux<P, T>;
  __host__ __device__ static type make(const double (&)[P::NV], double gam) { return type{T(gam)}; }
};
template <class P, class T>
struct FluxOf<P, T, true> {
  using type = DeviationFlux<P, T>;
  __host__ __device__ static type make(const double (&w0)[P::NV], double gam) {
    return type{P::make_ref(w0, gam), T(gam)};
  }
};

template <int ORDER, int FORM, class T, int NV = 5>
struct SchemeOf;
template <class T, int NV> struct SchemeOf<2, 0, T, NV> { using type = ader_gen::SchemeM2<T, NV>; };
template <class T, int NV> struct SchemeOf<2, 1, T, NV> { using type = ader_gen::SchemeN2<T, NV>; };
template <class T, int NV> struct SchemeOf<3, 0, T, NV> { using type = ader_gen::SchemeM3<T, NV>; };
template <class T, int NV> struct SchemeOf<3, 1, T, NV> { using type = ader_gen::SchemeN3<T, NV>; };
template <class T, int NV> struct SchemeOf<4, 0, T, NV> { using type = ader_gen::SchemeM4<T, NV>; };
template <class T, int NV> struct SchemeOf<4, 1, T, NV> { using type = ader_gen::SchemeN4<T, NV>; };

// Side SIDE's packet, rows SIDE*15 .. SIDE*15+14 of PK (u_b, <u>, <F>, each
// for the five variables); q walks the rows and is left at the next side.
template <class S, class T, int SIDE, class Phys, class Acc>
__host__ __device__ __forceinline__ void store_side(const T (&w)[S::LS][5], const T (&e)[S::NE][5],
                                                    const Phys& ph, Acc& acc, T*& q, long long N) {
  T ub[5], ua[5], fa[5];
  S::template side<SIDE>(w, e, ph, acc, ub, ua, fa);
#pragma unroll
  for (int v = 0; v < 5; ++v) { *q = ub[v]; q = next_row(q, N); }
#pragma unroll
  for (int v = 0; v < 5; ++v) { *q = ua[v]; q = next_row(q, N); }
#pragma unroll
  for (int v = 0; v < 5; ++v) { *q = fa[v]; q = next_row(q, N); }
}

// A scan that ignores the states handed to it.
struct NoScan {
  template <class U>
  __host__ __device__ void operator()(const U&) const {}
};

// ---------------------------------------------------------------------------
// Non-stiff source term (Euler): an affine S(u) = A u + b, the same for all
// zones of a context (row-major A: S_v = sum_q A[v][q] u_q + b_v).  At the
// predictor nodes the generated code takes the scaled source dt S from
// AffineSrc: in the point form dt (A u + b); in the deviation form dt A du of
// the deviation du, with base = dt S(zone average) (formed in double) for the
// constant part.  dt times the space-time average of S over the zone, the
// source term of eq. (6), is dt (A mean + b) with mean the space-time mean of
// the final polynomial, which for an affine S equals eq. (35), (44), (53)
// and (A.7), (B.6), (C.6).
// ---------------------------------------------------------------------------
struct SourceAffine {
  double A[25];
  double b[5];
};

template <class T, bool DEV>
struct AffineSrc {
  static constexpr bool kActive = true;
  const SourceAffine& s;
  T h;
  T base[5];
  __host__ __device__ AffineSrc(const SourceAffine& src, double dt, const double (&w0)[5])
      : s(src), h(T(dt)) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double a = s.b[v];
#pragma unroll
      for (int q = 0; q < 5; ++q) a += s.A[v * 5 + q] * w0[q];
      base[v] = DEV ? T(dt * a) : T(0);
    }
  }
  __host__ __device__ void operator()(const T (&u)[5], T (&out)[5]) const {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T a = DEV ? T(0) : T(s.b[v]);
#pragma unroll
      for (int q = 0; q < 5; ++q) a += T(s.A[v * 5 + q]) * u[q];
      out[v] = h * a;
    }
  }
};

// dt (A mean + b) for the final modes of a zone (SB row v at n)
template <class S, class T>
__host__ __device__ __forceinline__ void store_source_average(const SourceAffine& src, double dt,
                                                              const double (&w0)[5],
                                                              const T (&e)[S::NE][5],
                                                              double* __restrict__ SB, long long N,
                                                              long long n) {
  double m[5];
  S::mean_dev(e, m);
  double* q = SB + n;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double a = src.b[v];
#pragma unroll
    for (int k = 0; k < 5; ++k) a += src.A[v * 5 + k] * (w0[k] + m[k]);
    *q = dt * a;
    q = next_row(q, N);
  }
}

// Per zone: load the reconstruction, positivity scaling, space-time predictor
// (Sec. IV / App. A), positivity scaling, and the six face-side packets (in
// the deviation form without the zone-average part).  FUSED: the facial
// check set is scanned while the sides are formed (their states are that
// set), else in a pass of its own before them; the results are the same.
// SRC: with the affine source *src, whose dt-scaled space-time average goes
// to SB (rows of 5 doubles).
template <class T, int ORDER, int FORM, bool DEV, bool FUSED = true, bool SRC = false>
__host__ __device__ __forceinline__ void predict_zone_body(
    const double (&w0)[5], T (&w)[SchemeOf<ORDER, FORM, T>::type::LS][5], T* __restrict__ PK,
    const Grid& g, double h, double inv_dx, double inv_dy, double inv_dz, double gam, PosCtl pc,
    long long n, const SourceAffine* src, double* __restrict__ SB);

template <class T, int ORDER, int FORM, bool DEV, bool FUSED = true, bool SRC = false>
__host__ __device__ __forceinline__ void predict_zone(const double* __restrict__ U,
                                                      const T* __restrict__ W,
                                                      T* __restrict__ PK, const Grid& g,
                                                      double h, double inv_dx, double inv_dy,
                                                      double inv_dz, double gam, PosCtl pc,
                                                      long long n,
                                                      const SourceAffine* src = nullptr,
                                                      double* __restrict__ SB = nullptr) {
  using S = typename SchemeOf<ORDER, FORM, T>::type;
  constexpr int LS = S::LS;
  double w0[5];
  {
    const double* q = U + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) { w0[v] = *q; q = next_row(q, g.S); }
  }
  T w[LS][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[0][v] = DEV ? T(0) : T(w0[v]);
  {
    const T* q = W + n;
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) { w[m][v] = *q; q = next_row(q, g.S); }
  }
  predict_zone_body<T, ORDER, FORM, DEV, FUSED, SRC>(w0, w, PK, g, h, inv_dx, inv_dy, inv_dz, gam,
                                                     pc, n, src, SB);
}

// predict_zone with the zone's modes in LDS (mode m of variable v at
// sw[((m - 1) 5 + v) nz]), for the kernel that reconstructs in the same
// launch
template <class T, int ORDER, int FORM, bool DEV>
__device__ __forceinline__ void predict_zone_lds(const double* __restrict__ U, const T* sw, int nz,
                                                 T* __restrict__ PK, const Grid& g, double h,
                                                 double inv_dx, double inv_dy, double inv_dz,
                                                 double gam, PosCtl pc, long long n) {
  using S = typename SchemeOf<ORDER, FORM, T>::type;
  constexpr int LS = S::LS;
  double w0[5];
  {
    const double* q = U + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) { w0[v] = *q; q = next_row(q, g.S); }
  }
  T w[LS][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[0][v] = DEV ? T(0) : T(w0[v]);
#pragma unroll
  for (int m = 1; m < LS; ++m)
#pragma unroll
    for (int v = 0; v < 5; ++v) w[m][v] = sw[((m - 1) * 5 + v) * nz];
  predict_zone_body<T, ORDER, FORM, DEV, true, false>(w0, w, PK, g, h, inv_dx, inv_dy, inv_dz,
                                                      gam, pc, n, nullptr, nullptr);
}

template <class T, int ORDER, int FORM, bool DEV, bool FUSED, bool SRC>
__host__ __device__ __forceinline__ void predict_zone_body(
    const double (&w0)[5], T (&w)[SchemeOf<ORDER, FORM, T>::type::LS][5], T* __restrict__ PK,
    const Grid& g, double h, double inv_dx, double inv_dy, double inv_dz, double gam, PosCtl pc,
    long long n, const SourceAffine* src, double* __restrict__ SB) {
  static_assert(FUSED || !SRC, "the source instance has the fused facial check");
  using S = typename SchemeOf<ORDER, FORM, T>::type;
  constexpr int LS = S::LS, NE = S::NE;
  {
    PosScan<T, 5, DEV> scan(w0);
    S::spatial_points(w, scan);
    const double theta = scan.near ? theta_spatial_tab(w0, w, S::spatial_phi, gam, pc.limit) : 1.0;
    if (pos_scales(pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w[m][v] *= th;
    }
  }
  const auto ph = FluxOf<Euler<T>, T, DEV>::make(w0, gam);
  T e[NE][5];
  if constexpr (SRC)
    S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph,
               AffineSrc<T, DEV>(*src, h, w0));
  else
    S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
  if constexpr (!FUSED) {
    PosScan<T, 5, DEV> scan(w0);
    S::facial_points(w, e, scan);
    const double theta = scan.near ? theta_facial_tab(w0, w, e, S::facial_phi, gam, pc.limit) : 1.0;
    if (pos_scales(pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w[m][v] *= th;
#pragma unroll
      for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) e[m][v] *= th;
    }
    NoScan none;
    T* q = PK + n;
    store_side<S, T, 0>(w, e, ph, none, q, g.S);
    store_side<S, T, 1>(w, e, ph, none, q, g.S);
    store_side<S, T, 2>(w, e, ph, none, q, g.S);
    store_side<S, T, 3>(w, e, ph, none, q, g.S);
    store_side<S, T, 4>(w, e, ph, none, q, g.S);
    store_side<S, T, 5>(w, e, ph, none, q, g.S);
    return;
  }
  // The six face-side packets.  The states they evaluate are the facial
  // check set of the positivity safeguard and are scanned on the way; in the
  // rare zone the scan flags, theta comes from the exact pass and the sides
  // are formed again from the scaled polynomial (the same result as scaling
  // before forming them).
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    PosScan<T, 5, DEV> scan(w0);
    T* q = PK + n;
    store_side<S, T, 0>(w, e, ph, scan, q, g.S);
    store_side<S, T, 1>(w, e, ph, scan, q, g.S);
    store_side<S, T, 2>(w, e, ph, scan, q, g.S);
    store_side<S, T, 3>(w, e, ph, scan, q, g.S);
    store_side<S, T, 4>(w, e, ph, scan, q, g.S);
    store_side<S, T, 5>(w, e, ph, scan, q, g.S);
    if (pass == 1 || !scan.near) break;
    const double theta = theta_facial_tab(w0, w, e, S::facial_phi, gam, pc.limit);
    if (!pos_scales(pc, theta)) break;
    const T th = T(theta);
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) w[m][v] *= th;
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) e[m][v] *= th;
  }
  // the source term of eq. (6) from the final (possibly scaled) polynomial
  if constexpr (SRC) store_source_average<S, T>(*src, h, w0, e, SB, g.S, n);
}

// An SSP-RK stage (Sec. II.d; Euler): the predictor is bypassed, so a zone
// loads its reconstruction, applies the spatial positivity scaling (whose
// check set holds every point the RK side packets evaluate) and writes the
// six side packets of its spatial polynomial at the stage time, in the
// layout the face-flux kernel reads.
template <class T, int ORDER, bool DEV>
__host__ __device__ __forceinline__ void rk_sides_zone(const double* __restrict__ U,
                                                       const T* __restrict__ W,
                                                       T* __restrict__ PK, const Grid& g,
                                                       double gam, PosCtl pc, long long n) {
  using S = typename SchemeOf<ORDER, 0, T>::type;
  constexpr int LS = S::LS;
  double w0[5];
  {
    const double* q = U + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) { w0[v] = *q; q = next_row(q, g.S); }
  }
  T w[LS][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[0][v] = DEV ? T(0) : T(w0[v]);
  {
    const T* q = W + n;
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) { w[m][v] = *q; q = next_row(q, g.S); }
  }
  {
    PosScan<T, 5, DEV> scan(w0);
    S::spatial_points(w, scan);
    const double theta = scan.near ? theta_spatial_tab(w0, w, S::spatial_phi, gam, pc.limit) : 1.0;
    if (pos_scales(pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w[m][v] *= th;
    }
  }
  const auto ph = FluxOf<Euler<T>, T, DEV>::make(w0, gam);
  NoScan none;
  T* q = PK + n;
  auto side = [&](auto side_c) {
    constexpr int SIDE = decltype(side_c)::value;
    T ub[5], ua[5], fa[5];
    S::template side_rk<SIDE>(w, ph, none, ub, ua, fa);
#pragma unroll
    for (int v = 0; v < 5; ++v) { *q = ub[v]; q = next_row(q, g.S); }
#pragma unroll
    for (int v = 0; v < 5; ++v) { *q = ua[v]; q = next_row(q, g.S); }
#pragma unroll
    for (int v = 0; v < 5; ++v) { *q = fa[v]; q = next_row(q, g.S); }
  };
  side(std::integral_constant<int, 0>{});
  side(std::integral_constant<int, 1>{});
  side(std::integral_constant<int, 2>{});
  side(std::integral_constant<int, 3>{});
  side(std::integral_constant<int, 4>{});
  side(std::integral_constant<int, 5>{});
}

// One SSP-RK stage combination (eq. 18-20) in double, with L(U) = -sum_d
// (F_{i+1/2} - F_{i-1/2}) / dx_d from the fluxes of the current stage state:
//   U <- a_n Un + a_c U + c_l h L + a_2 S2 + a_3 S3 + c_d D3
// (terms with a zero weight are not read).  save_state receives the result
// and save_hl receives h L, for the later stages of (20) that reuse them.
struct RkStage {
  double a_n, a_c, c_l, a_2, a_3, c_d;
  const double* Un;
  const double* S2;
  const double* S3;
  const double* D3;
  double* save_state;
  double* save_hl;
};

// The same combination for the MHD face fields, their rate L_B = -curl E
// (eq. 8 per unit time; B_d at the lower d-face, E_c at the lower c-edge).
__host__ __device__ __forceinline__ void rk_stage_field_zone(double* __restrict__ B,
                                                             const double* __restrict__ E,
                                                             const RkStage& st, const Grid& g,
                                                             double h, double dx, double dy,
                                                             double dz, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long px = zone_of(wrap(i + 1, g.nx), j, k, g);
  const long long py = zone_of(i, wrap(j + 1, g.ny), k, g);
  const long long pz = zone_of(i, j, wrap(k + 1, g.nz), g);
  const double* Ex = E;
  const double* Ey = E + g.S;
  const double* Ez = E + 2 * g.S;
  const double curl[3] = {(Ez[py] - Ez[n]) / dy - (Ey[pz] - Ey[n]) / dz,
                          (Ex[pz] - Ex[n]) / dz - (Ez[px] - Ez[n]) / dx,
                          (Ey[px] - Ey[n]) / dx - (Ex[py] - Ex[n]) / dy};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long at = (long long)c * g.S + n;
    const double hl = -(h * curl[c]);
    double b = st.a_c * B[at];
    if (st.a_n != 0.0) b = st.a_n * st.Un[at] + b;
    b = b + st.c_l * hl;
    if (st.a_2 != 0.0) b = b + st.a_2 * st.S2[at];
    if (st.a_3 != 0.0) b = b + st.a_3 * st.S3[at];
    if (st.c_d != 0.0) b = b + st.c_d * st.D3[at];
    if (st.save_hl) st.save_hl[at] = hl;
    if (st.save_state) st.save_state[at] = b;
    B[at] = b;
  }
}

__host__ __device__ __forceinline__ void rk_stage_zone(double* __restrict__ U,
                                                       const double* __restrict__ F,
                                                       const RkStage& st, const Grid& g,
                                                       double h, double dx, double dy,
                                                       double dz, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long up[3] = {zone_of(wrap(i + 1, g.nx), j, k, g), zone_of(i, wrap(j + 1, g.ny), k, g),
                           zone_of(i, j, wrap(k + 1, g.nz), g)};
  const double inv[3] = {1.0 / dx, 1.0 / dy, 1.0 / dz};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long at = (long long)v * g.S + n;
    double l = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double fp = F[((long long)ax * 5 + v) * g.S + up[ax]];
      const double fm = F[((long long)ax * 5 + v) * g.S + n];
      l = l - (fp - fm) * inv[ax];
    }
    const double hl = h * l;
    double u = st.a_c * U[at];
    if (st.a_n != 0.0) u = st.a_n * st.Un[at] + u;
    u = u + st.c_l * hl;
    if (st.a_2 != 0.0) u = u + st.a_2 * st.S2[at];
    if (st.a_3 != 0.0) u = u + st.a_3 * st.S3[at];
    if (st.c_d != 0.0) u = u + st.c_d * st.D3[at];
    if (st.save_hl) st.save_hl[at] = hl;
    if (st.save_state) st.save_state[at] = u;
    U[at] = u;
  }
}

// ---------------------------------------------------------------------------
// Riemann fluxes at the faces (Sec. II.3, V): wave structure frozen at the
// two barycentre states.
// ---------------------------------------------------------------------------
// The face solvers contract multiply-adds within each expression only
// (fp contract on): their rounding then does not depend on the code a kernel
// inlines them into (which products it shares with other faces), so the
// fused face-flux+update kernel and the two-kernel path give equal bits.
//
// Euler pressure and physical flux along AXIS, as Euler<T>::pressure and
// Euler<T>::flux, for the face solvers.
template <class T>
__host__ __device__ __forceinline__ T face_pressure(const T (&u)[5], T gam) {
#pragma clang fp contract(on)
  return (gam - T(1)) * (u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
}

template <int AXIS>
__host__ __device__ __forceinline__ void face_average_flux(const double (&u)[5], double (&f)[5],
                                                           double gam) {
#pragma clang fp contract(on)
  const double rinv = 1.0 / u[0];
  const double vn = u[1 + AXIS] * rinv;
  const double ke = 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * rinv;
  const double p = (gam - 1.0) * (u[4] - ke);
  f[0] = u[1 + AXIS];
  f[1] = u[1] * vn;
  f[2] = u[2] * vn;
  f[3] = u[3] * vn;
  f[1 + AXIS] += p;
  f[4] = (u[4] + p) * vn;
}

// HLL combination (eq. 17 / 56) with signal speeds lam_l <= 0 <= lam_r.
template <class T, int NV>
__host__ __device__ __forceinline__ void hll_combine(T lam_l, T lam_r, const T (&ul)[NV],
                                                     const T (&fl)[NV], const T (&ur)[NV],
                                                     const T (&fr)[NV], T (&out)[NV]) {
#pragma clang fp contract(on)
  const T inv = T(1) / (lam_r - lam_l);
#pragma unroll
  for (int v = 0; v < NV; ++v)
    out[v] = (lam_r * fl[v] - lam_l * fr[v] + lam_r * lam_l * (ur[v] - ul[v])) * inv;
}

// Linearized flux: (F_L + F_R)/2 - R |Lambda| L (u_R - u_L)/2 with the Euler
// eigen-system at the mean of the two barycentre primitive states.
template <class T, int AXIS>
__host__ __device__ __forceinline__ void linearized_flux(const T (&ubl)[5], const T (&ul)[5], const T (&fl)[5],
                                                const T (&ubr)[5], const T (&ur)[5], const T (&fr)[5],
                                                T gam, T (&out)[5]) {
#pragma clang fp contract(on)
  constexpr int A = 1 + AXIS;
  constexpr int B = AXIS == 0 ? 2 : 1;
  constexpr int C = AXIS == 2 ? 2 : 3;
  const T rl = ubl[0], rr = ubr[0];
  const T pl = face_pressure(ubl, gam), pr = face_pressure(ubr, gam);
  const T rho = T(0.5) * (rl + rr);
  const T vn = T(0.5) * (ubl[A] / rl + ubr[A] / rr);
  const T va = T(0.5) * (ubl[B] / rl + ubr[B] / rr);
  const T vb = T(0.5) * (ubl[C] / rl + ubr[C] / rr);
  const T p = T(0.5) * (pl + pr);
  const T c2 = gam * p / rho;
  const T c = sqrt(c2);
  const T q2 = vn * vn + va * va + vb * vb;
  const T hent = c2 / (gam - T(1)) + T(0.5) * q2;
  const T d1 = ur[0] - ul[0], dn = ur[A] - ul[A], da = ur[B] - ul[B], db = ur[C] - ul[C];
  const T de = ur[4] - ul[4];
  const T a_a = da - va * d1;
  const T a_b = db - vb * d1;
  const T de_bar = de - a_a * va - a_b * vb;
  const T a2 = (gam - T(1)) / c2 * (d1 * (hent - vn * vn) + vn * dn - de_bar);
  const T a1 = (d1 * (vn + c) - dn - c * a2) / (T(2) * c);
  const T a5 = d1 - a1 - a2;
  const T w1 = fabs(vn - c) * a1, w2 = fabs(vn) * a2, w5 = fabs(vn + c) * a5;
  const T wa = fabs(vn) * a_a, wb = fabs(vn) * a_b;
  T dis[5];
  const T s = w1 + w2 + w5;
  dis[0] = s;
  dis[A] = w1 * (vn - c) + w2 * vn + w5 * (vn + c);
  dis[B] = s * va + wa;
  dis[C] = s * vb + wb;
  dis[4] = w1 * (hent - vn * c) + w2 * T(0.5) * q2 + wa * va + wb * vb + w5 * (hent + vn * c);
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = T(0.5) * (fl[v] + fr[v]) - T(0.5) * dis[v];
}

// Flux at the lower AXIS-face of zone n from the packets of the upper side of
// zone nl and the lower side of zone n.  Deviation form: the packets hold
// differences from the zone averages wl, wr (double), and both solvers are
// affine in (u_L, u_R, F_L, F_R) for frozen wave speeds / eigen-system, so
// the flux splits exactly into the solver applied to the zone averages (in
// double: HLL (lr F(wl) - ll F(wr))/(lr - ll) with the jump term moved to the
// FP32 part, linearized (F(wl) + F(wr))/2) plus the solver applied to the
// deviations with the jump wr - wl added to the right state (FP32).
template <class T, int RS, int AXIS, bool DEV>
__host__ __device__ __forceinline__ void face_flux_values(const double* __restrict__ U,
                                                          const T* __restrict__ PK,
                                                          const Grid& g, long long n,
                                                          long long nl, double gam,
                                                          double (&res)[5]) {
#pragma clang fp contract(on)
  T ubl[5], ul[5], fl[5], ubr[5], ur[5], fr[5], out[5];
  double wl[5], wr[5];
  constexpr int SL = 2 * AXIS + 1, SR = 2 * AXIS;  // top side of the lower zone, bottom side of this
  {
    const T* ql = PK + (long long)(SL * 15) * g.S + nl;
    const T* qr = PK + (long long)(SR * 15) * g.S + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      ubl[v] = *ql; ql = next_row(ql, g.S);
      ubr[v] = *qr; qr = next_row(qr, g.S);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      ul[v] = *ql; ql = next_row(ql, g.S);
      ur[v] = *qr; qr = next_row(qr, g.S);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      fl[v] = *ql; ql = next_row(ql, g.S);
      fr[v] = *qr; qr = next_row(qr, g.S);
    }
  }
  if constexpr (DEV) {
    const double* pl = U + nl;
    const double* pr = U + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      wl[v] = *pl; pl = next_row(pl, g.S);
      wr[v] = *pr; pr = next_row(pr, g.S);
      ubl[v] += T(wl[v]);
      ubr[v] += T(wr[v]);
      ur[v] += T(wr[v] - wl[v]);
    }
  }
  const T tg = T(gam);
  if constexpr (RS == 0) {
    // signal speeds of the barycentre states
    const T il = recip(ubl[0]), ir = recip(ubr[0]);
    const T vl = ubl[1 + AXIS] * il, vr = ubr[1 + AXIS] * ir;
    const T cl = fsqrt(tg * face_pressure(ubl, tg) * il);
    const T cr = fsqrt(tg * face_pressure(ubr, tg) * ir);
    const T lam_l = fmin(fmin(vl - cl, vr - cr), T(0));
    const T lam_r = fmax(fmax(vl + cl, vr + cr), T(0));
    hll_combine<T, 5>(lam_l, lam_r, ul, fl, ur, fr, out);
    if constexpr (DEV) {
      double Fl[5], Fr[5];
      face_average_flux<AXIS>(wl, Fl, gam);
      face_average_flux<AXIS>(wr, Fr, gam);
      const double ll = lam_l, lr = lam_r, inv = 1.0 / (lr - ll);
#pragma unroll
      for (int v = 0; v < 5; ++v) res[v] = (lr * Fl[v] - ll * Fr[v]) * inv + double(out[v]);
      return;
    }
  } else {
    linearized_flux<T, AXIS>(ubl, ul, fl, ubr, ur, fr, tg, out);
    if constexpr (DEV) {
      double Fl[5], Fr[5];
      face_average_flux<AXIS>(wl, Fl, gam);
      face_average_flux<AXIS>(wr, Fr, gam);
#pragma unroll
      for (int v = 0; v < 5; ++v) res[v] = 0.5 * (Fl[v] + Fr[v]) + double(out[v]);
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) res[v] = double(out[v]);
}

template <class T, int RS, int AXIS, bool DEV>
__host__ __device__ __forceinline__ void face_flux_axis(const double* __restrict__ U,
                                                        const T* __restrict__ PK,
                                                        double* __restrict__ F, const Grid& g,
                                                        long long n, long long nl, double gam) {
  double res[5];
  face_flux_values<T, RS, AXIS, DEV>(U, PK, g, n, nl, gam, res);
  double* qf = F + (long long)(AXIS * 5) * g.S + n;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    *qf = res[v];
    qf = next_row(qf, g.S);
  }
}

// Each face flux is formed once, by the zone above it, so both zones that
// share a face see the same value and the update conserves exactly.
template <class T, int RS, bool DEV>
__host__ __device__ __forceinline__ void face_flux_zone(const double* __restrict__ U,
                                                        const T* __restrict__ PK,
                                                        double* __restrict__ F, const Grid& g,
                                                        double gam, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  face_flux_axis<T, RS, 0, DEV>(U, PK, F, g, n, zone_of(wrap(i - 1, g.nx), j, k, g), gam);
  face_flux_axis<T, RS, 1, DEV>(U, PK, F, g, n, zone_of(i, wrap(j - 1, g.ny), k, g), gam);
  face_flux_axis<T, RS, 2, DEV>(U, PK, F, g, n, zone_of(i, j, wrap(k - 1, g.nz), g), gam);
}

// ---------------------------------------------------------------------------
// Linear advection of five components, F_d(u) = a_d u: the test system on
// which the scheme translates any data exactly at unit Courant number.  The
// same predictor and face quadrature run with the linear flux (point form,
// no positivity handling), and the face flux is the upwind limit of the HLL
// flux of eq. (56), whose signal speeds are min(a_d, 0) and max(a_d, 0).
// ---------------------------------------------------------------------------
template <class T>
struct AdvFlux {
  static constexpr bool kDeviation = false;
  static constexpr int comp(int c) { return c; }
  T a[3];
  template <int AXIS, int NV>
  __host__ __device__ inline void flux(const T (&u)[NV], T (&f)[NV]) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) f[v] = a[AXIS] * u[v];
  }
};

template <class T, int ORDER, int FORM>
__host__ __device__ __forceinline__ void predict_zone_adv(const double* __restrict__ U,
                                                          const T* __restrict__ W,
                                                          T* __restrict__ PK, const Grid& g,
                                                          double h, double inv_dx, double inv_dy,
                                                          double inv_dz, double ax, double ay,
                                                          double az, long long n) {
  using S = typename SchemeOf<ORDER, FORM, T>::type;
  constexpr int LS = S::LS, NE = S::NE;
  T w[LS][5];
  {
    const double* q = U + n;
#pragma unroll
    for (int v = 0; v < 5; ++v) { w[0][v] = T(*q); q = next_row(q, g.S); }
  }
  {
    const T* q = W + n;
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) { w[m][v] = *q; q = next_row(q, g.S); }
  }
  const AdvFlux<T> ph{{T(ax), T(ay), T(az)}};
  T e[NE][5];
  S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
  NoScan none;
  T* q = PK + n;
  store_side<S, T, 0>(w, e, ph, none, q, g.S);
  store_side<S, T, 1>(w, e, ph, none, q, g.S);
  store_side<S, T, 2>(w, e, ph, none, q, g.S);
  store_side<S, T, 3>(w, e, ph, none, q, g.S);
  store_side<S, T, 4>(w, e, ph, none, q, g.S);
  store_side<S, T, 5>(w, e, ph, none, q, g.S);
}

// Flux at the lower AXIS-face of zone n: the upper side's face-averaged
// flux of the lower zone nl for a > 0, this zone's lower side's for a < 0.
template <class T, int AXIS>
__host__ __device__ __forceinline__ void face_flux_adv_axis(const T* __restrict__ PK,
                                                            double* __restrict__ F, const Grid& g,
                                                            long long n, long long nl, double a) {
  constexpr int SL = 2 * AXIS + 1, SR = 2 * AXIS;
  double* qf = F + (long long)(AXIS * 5) * g.S + n;
  const T* q = a > 0.0 ? PK + (long long)(SL * 15 + 10) * g.S + nl
                       : PK + (long long)(SR * 15 + 10) * g.S + n;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    *qf = a != 0.0 ? double(*q) : 0.0;
    qf = next_row(qf, g.S);
    q = next_row(q, g.S);
  }
}

template <class T>
__host__ __device__ __forceinline__ void face_flux_adv_zone(const T* __restrict__ PK,
                                                            double* __restrict__ F, const Grid& g,
                                                            double ax, double ay, double az,
                                                            long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  face_flux_adv_axis<T, 0>(PK, F, g, n, zone_of(wrap(i - 1, g.nx), j, k, g), ax);
  face_flux_adv_axis<T, 1>(PK, F, g, n, zone_of(i, wrap(j - 1, g.ny), k, g), ay);
  face_flux_adv_axis<T, 2>(PK, F, g, n, zone_of(i, j, wrap(k - 1, g.nz), g), az);
}

// eq. (6) in double: U -= dt/dx (F_{i+1/2} - F_{i-1/2}) + ... (y, z)
__host__ __device__ __forceinline__ void update_zone(double* __restrict__ U, const double* __restrict__ F,
                                                     const Grid& g, double h, double dx,
                                                     double dy, double dz, long long n) {
#pragma clang fp contract(on)   // as the fused kernel's update: equal bits
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long up[3] = {zone_of(wrap(i + 1, g.nx), j, k, g), zone_of(i, wrap(j + 1, g.ny), k, g),
                           zone_of(i, j, wrap(k + 1, g.nz), g)};
  const double c[3] = {h / dx, h / dy, h / dz};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double u = U[(long long)v * g.S + n];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double fp = F[((long long)ax * 5 + v) * g.S + up[ax]];
      const double fm = F[((long long)ax * 5 + v) * g.S + n];
      u = u - c[ax] * (fp - fm);
    }
    U[(long long)v * g.S + n] = u;
  }
}

// eq. (6) with the source term: update_zone, then + dt S-bar (SB rows)
__host__ __device__ __forceinline__ void source_zone(double* __restrict__ U,
                                                     const double* __restrict__ SB, const Grid& g,
                                                     long long n) {
#pragma unroll
  for (int v = 0; v < 5; ++v) U[(long long)v * g.S + n] += SB[(long long)v * g.S + n];
}

// ---------------------------------------------------------------------------
// dt by CFL: per zone sum_d (|v_d| + c) / dx_d; wavefront then block maximum
// into one partial per block; a single block reduces the partials.
// ---------------------------------------------------------------------------
// sum_d (|v_d| + c) / dx_d of one zone; flags rho <= 0, P <= 0 or non-finite
__host__ __device__ __forceinline__ double dt_rate_zone(const double* __restrict__ U, const Grid& g,
                                                        double gam, double dx, double dy, double dz,
                                                        long long n, int& isbad) {
  const double r = U[n];
  const double m[3] = {U[g.S + n], U[2 * g.S + n], U[3 * g.S + n]};
  const double E = U[4 * g.S + n];
  const double p = (gam - 1.0) * (E - 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / r);
  const bool ok = r > 0.0 && p > 0.0 && __builtin_isfinite(r) && __builtin_isfinite(p) && __builtin_isfinite(m[0]) &&
                  __builtin_isfinite(m[1]) && __builtin_isfinite(m[2]);
  if (!ok) {
    isbad = 1;
    return 0.0;
  }
  const double c = sqrt(gam * p / r);
  return (fabs(m[0] / r) + c) / dx + (fabs(m[1] / r) + c) / dy + (fabs(m[2] / r) + c) / dz;
}

// ---------------------------------------------------------------------------
// Ideal MHD.  Face layout: B[d][n] is B_d on the lower d-face of zone n; the
// zone field b_0 is B0[d][n] (double), the normal moments of Sec. III are
// BN[a-1][d][n], the modes of the remaining reconstruction WB[m-1][d][n].
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ long long shifted(const Grid& g, int i, int j, int k, int axis,
                                                      int o) {
  if (axis == 0) return zone_of(wrap(i + o, g.nx), j, k, g);
  if (axis == 1) return zone_of(i, wrap(j + o, g.ny), k, g);
  return zone_of(i, j, wrap(k + o, g.nz), g);
}

// Sec. III: each component's zone average and normal moments from its own
// faces.  f[q] is the face at offset q - 1/2 from the zone centre (q = -2..3).
// Order 2: mean and difference; order 3: stencils of eq. (22)-(23),
// smoothness eq. (24), equal linear weights; order 4: eq. (26)-(28),
// smoothness eq. (29), linear weights (1, 100, 1).
template <class T, int M>
__host__ __device__ __forceinline__ void bface_zone(const double* __restrict__ B,
                                                    double* __restrict__ B0, T* __restrict__ BN,
                                                    const Grid& g, long long n) {
  constexpr double kEps = 1.0e-12;
  int i, j, k;
  zone_ijk(g, n, i, j, k);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double f[6];  // offsets -2 .. 3
#pragma unroll
    for (int q = -2; q <= 3; ++q) {
      const bool need = (M == 2 && q >= 0 && q <= 1) || (M == 3 && q >= -1 && q <= 2) || M == 4;
      f[q + 2] = need ? B[(long long)d * g.S + shifted(g, i, j, k, d, q)] : 0.0;
    }
    const double fm25 = f[0], fm15 = f[1], fm05 = f[2], fp05 = f[3], fp15 = f[4], fp25 = f[5];
    double b[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (M == 2) {
      b[0] = 0.5 * (fm05 + fp05);
      b[1] = fp05 - fm05;
    } else if constexpr (M == 3) {
      const double s1[3] = {(8.0 * fm05 - fm15 + 5.0 * fp05) / 12.0, fp05 - fm05,
                            (fp05 + fm15 - 2.0 * fm05) / 2.0};
      const double s2[3] = {(8.0 * fp05 - fp15 + 5.0 * fm05) / 12.0, fp05 - fm05,
                            (fm05 + fp15 - 2.0 * fp05) / 2.0};
      const double i1 = s1[1] * s1[1] + 13.0 * s1[2] * s1[2] / 3.0;
      const double i2 = s2[1] * s2[1] + 13.0 * s2[2] * s2[2] / 3.0;
      const double a1 = 1.0 / ((kEps + i1) * (kEps + i1)), a2 = 1.0 / ((kEps + i2) * (kEps + i2));
      const double tot = a1 + a2;
#pragma unroll
      for (int q = 0; q < 3; ++q) b[q] = (a1 * s1[q] + a2 * s2[q]) / tot;
    } else {
      const double s[3][4] = {
          {(9.0 * fp05 + 19.0 * fm05 - 5.0 * fm15 + fm25) / 24.0,
           (59.0 * fp05 - 57.0 * fm05 - 3.0 * fm15 + fm25) / 60.0,
           (3.0 * fp05 - 7.0 * fm05 + 5.0 * fm15 - fm25) / 4.0,
           (fp05 - 3.0 * fm05 + 3.0 * fm15 - fm25) / 6.0},
          {(-fp15 + 13.0 * fp05 + 13.0 * fm05 - fm15) / 24.0,
           (-fp15 + 63.0 * fp05 - 63.0 * fm05 + fm15) / 60.0,
           (fp15 - fp05 - fm05 + fm15) / 4.0,
           (fp15 - 3.0 * fp05 + 3.0 * fm05 - fm15) / 6.0},
          {(fp25 - 5.0 * fp15 + 19.0 * fp05 + 9.0 * fm05) / 24.0,
           (-fp25 + 3.0 * fp15 + 57.0 * fp05 - 59.0 * fm05) / 60.0,
           (-fp25 + 5.0 * fp15 - 7.0 * fp05 + 3.0 * fm05) / 4.0,
           (fp25 - 3.0 * fp15 + 3.0 * fp05 - fm05) / 6.0}};
      double a[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double t = s[q][1] + 0.1 * s[q][3];
        const double is = t * t + 13.0 * s[q][2] * s[q][2] / 3.0 + 781.0 * s[q][3] * s[q][3] / 20.0;
        a[q] = (q == 1 ? 100.0 : 1.0) / ((kEps + is) * (kEps + is));
      }
      const double tot = a[0] + a[1] + a[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = (a[0] * s[0][q] + a[1] * s[1][q] + a[2] * s[2][q]) / tot;
    }
    B0[(long long)d * g.S + n] = b[0];
#pragma unroll
    for (int a = 1; a < M; ++a) BN[((long long)(a - 1) * 3 + d) * g.S + n] = T(b[a]);
  }
}

// MHD side packet, kMhdSlots values per side: barycentre state (0-7), face
// averages of u (8-15) and F (16-23), on each edge q = 2 w + (side > 0) the
// edge average of the field flux of the component along transverse axis t_w
// (24 + q) and the edge averages of u (28 + 8 q + v).  The HLL flux reads
// only the field component of the edge states, the linearized flux all.
constexpr int kMhdSlots = 60;
__host__ __device__ constexpr int mhd_fe_slot(int q) { return 24 + q; }
__host__ __device__ constexpr int mhd_ue_slot(int q, int v) { return 28 + 8 * q + v; }
__host__ __device__ constexpr int mhd_edge_comp(int axis, int q) {
  return 5 + (q < 2 ? (axis == 0 ? 1 : 0) : (axis == 2 ? 1 : 2));
}

// EDGES_ALL: store every variable's edge average (linearized flux), else only
// the field component each edge needs (HLL)
template <class S, class T, int SIDE, bool EDGES_ALL, class Phys, class Acc>
__host__ __device__ __forceinline__ void store_side_mhd(const T (&w)[S::LS][8], const T (&e)[S::NE][8],
                                                        const Phys& ph, Acc& acc, T* __restrict__ PK,
                                                        long long N, long long n) {
  T ub[8], ua[8], fa[8], ue[4], fe[4];
  S::template side_edges<SIDE>(w, e, ph, acc, ub, ua, fa, ue, fe);
  RowCursor<T> r(PK, N, n, SIDE * kMhdSlots);
#pragma unroll
  for (int v = 0; v < 8; ++v) r.row(SIDE * kMhdSlots + v) = ub[v];
#pragma unroll
  for (int v = 0; v < 8; ++v) r.row(SIDE * kMhdSlots + 8 + v) = ua[v];
#pragma unroll
  for (int v = 0; v < 8; ++v) r.row(SIDE * kMhdSlots + 16 + v) = fa[v];
#pragma unroll
  for (int q = 0; q < 4; ++q) r.row(SIDE * kMhdSlots + mhd_fe_slot(q)) = fe[q];
  if constexpr (EDGES_ALL) {
    T ues[4][8];
    S::template edge_states<SIDE, Phys::kDeviation>(w, e, ues);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 8; ++v) r.row(SIDE * kMhdSlots + mhd_ue_slot(q, v)) = ues[q][v];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      r.row(SIDE * kMhdSlots + mhd_ue_slot(q, mhd_edge_comp(SIDE / 2, q))) = ue[q];
  }
}

// Per zone (MHD): hydro modes from U/W, field modes from B0/WB with the
// Sec. III normal moments BN on the pure-normal slots, positivity scaling,
// predictor, positivity scaling and the six side packets of 32 values
// (barycentre state, face averages of u and F, edge averages of u and F of
// the field component along each edge's transverse axis).
// RK: an SSP-RK stage (Sec. II.d): the predictor is bypassed (the
// evolutionary modes are a constant zero, so coinciding face points fold
// together) and the spatial check set, which holds every face point, is the
// only positivity check.
template <class T, int ORDER, int FORM, bool DEV, bool FUSED = true, bool EDGES_ALL = false,
          bool RK = false>
__host__ __device__ __forceinline__ void predict_zone_mhd(
    const double* __restrict__ U, const T* __restrict__ W, const double* __restrict__ B0,
    const T* __restrict__ WB, const T* __restrict__ BN, T* __restrict__ PK, const Grid& g,
    double h, double inv_dx, double inv_dy, double inv_dz, double gam, PosCtl pc, long long n) {
  using S = typename SchemeOf<ORDER, FORM, T, 8>::type;
  constexpr int LS = S::LS, NE = S::NE;
  double w0[8];
  {
    RowCursor<const double> ru(U, g.S, n), rb(B0, g.S, n);
#pragma unroll
    for (int v = 0; v < 5; ++v) w0[v] = ru.row(v);
#pragma unroll
    for (int c = 0; c < 3; ++c) w0[5 + c] = rb.row(c);
  }
  T w[LS][8];
#pragma unroll
  for (int v = 0; v < 8; ++v) w[0][v] = DEV ? T(0) : T(w0[v]);
  {
    RowCursor<const T> rw(W, g.S, n), rf(WB, g.S, n), rn(BN, g.S, n);
#pragma unroll
    for (int m = 1; m < LS; ++m) {
#pragma unroll
      for (int v = 0; v < 5; ++v) w[m][v] = rw.row((m - 1) * 5 + v);
#pragma unroll
      for (int c = 0; c < 3; ++c) w[m][5 + c] = rf.row((m - 1) * 3 + c);
    }
#pragma unroll
    for (int a = 1; a < ORDER; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int m = spatial_mode(c == 0 ? a : 0, c == 1 ? a : 0, c == 2 ? a : 0);
        w[m][5 + c] = rn.row((a - 1) * 3 + c);
      }
  }
  {
    PosScan<T, 8, DEV> scan(w0);
    S::spatial_points_all(w, scan);
    const double theta =
        scan.near ? theta_spatial_tab(w0, w, S::spatial_phi_all, gam, pc.limit) : 1.0;
    if (pos_scales(pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 8; ++v) w[m][v] *= th;
    }
  }
  const auto ph = FluxOf<Mhd<T>, T, DEV>::make(w0, gam);
  if constexpr (RK) {
    constexpr T ez[NE][8] = {};
    NoScan none;
    store_side_mhd<S, T, 0, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 1, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 2, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 3, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 4, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 5, EDGES_ALL>(w, ez, ph, none, PK, g.S, n);
    return;
  }
  T e[NE][8];
  S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
  if constexpr (!FUSED) {
    PosScan<T, 8, DEV> scan(w0);
    S::facial_points_all(w, e, scan);
    const double theta =
        scan.near ? theta_facial_tab(w0, w, e, S::facial_phi_all, gam, pc.limit) : 1.0;
    if (pos_scales(pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 8; ++v) w[m][v] *= th;
#pragma unroll
      for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int v = 0; v < 8; ++v) e[m][v] *= th;
    }
    NoScan none;
    store_side_mhd<S, T, 0, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 1, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 2, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 3, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 4, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    store_side_mhd<S, T, 5, EDGES_ALL>(w, e, ph, none, PK, g.S, n);
    return;
  }
  // side packets with the facial scan on the way, as in predict_zone
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    PosScan<T, 8, DEV> scan(w0);
    store_side_mhd<S, T, 0, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    store_side_mhd<S, T, 1, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    store_side_mhd<S, T, 2, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    store_side_mhd<S, T, 3, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    store_side_mhd<S, T, 4, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    store_side_mhd<S, T, 5, EDGES_ALL>(w, e, ph, scan, PK, g.S, n);
    if (pass == 1 || !scan.near) break;
    const double theta = theta_facial_tab(w0, w, e, S::facial_phi_all, gam, pc.limit);
    if (!pos_scales(pc, theta)) break;
    const T th = T(theta);
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int v = 0; v < 8; ++v) w[m][v] *= th;
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
      for (int v = 0; v < 8; ++v) e[m][v] *= th;
  }
}

// Riemann flux at the lower AXIS-face of zone n (MHD): the five hydro fluxes,
// and the same solver, with this face's speeds (HLL) or frozen eigen-system
// (linearized), applied to the edge states (eq. 57) on its four edges, of
// which the induction flux of the edge's field component enters the edge
// field.  Deviation form as for Euler: the solver applied to the zone
// averages (double) plus the solver applied to the deviations (FP32); on the
// edges the zone-average part is the field component of the same double
// flux.
template <class T, int RS, int AXIS, bool DEV>
__host__ __device__ __forceinline__ void face_flux_axis_mhd(const double* __restrict__ U,
                                                            const double* __restrict__ B0,
                                                            const T* __restrict__ PK,
                                                            double* __restrict__ F,
                                                            double* __restrict__ FE,
                                                            const Grid& g, long long n,
                                                            long long nl, double gam) {
  constexpr int SL = 2 * AXIS + 1, SR = 2 * AXIS;
  constexpr int l0 = SL * kMhdSlots, r0 = SR * kMhdSlots;   // first rows of the two sides
  RowCursor<const T> L(PK, g.S, nl, l0), R(PK, g.S, n, r0);
  double wl[8], wr[8];
  if constexpr (DEV) {
    RowCursor<const double> ul_(U, g.S, nl), ur_(U, g.S, n), bl_(B0, g.S, nl), br_(B0, g.S, n);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      wl[v] = ul_.row(v);
      wr[v] = ur_.row(v);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      wl[5 + c] = bl_.row(c);
      wr[5 + c] = br_.row(c);
    }
  }
  T ubl[8], ubr[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    ubl[v] = L.row(l0 + v);
    ubr[v] = R.row(r0 + v);
    if constexpr (DEV) {
      ubl[v] += T(wl[v]);
      ubr[v] += T(wr[v]);
    }
  }
  RowCursor<double> rf(F, g.S, n, AXIS * 5), re(FE, g.S, n, AXIS * 4);
  const T tg = T(gam);
  T out[5], eout[4];
  if constexpr (RS == 0) {
    const T il = recip(ubl[0]), ir = recip(ubr[0]);
    const T vl = ubl[1 + AXIS] * il, vr = ubr[1 + AXIS] * ir;
    const T cl = Mhd<T>::template fast_speed<AXIS>(ubl, tg);
    const T cr = Mhd<T>::template fast_speed<AXIS>(ubr, tg);
    const T lam_l = fmin(fmin(vl - cl, vr - cr), T(0));
    const T lam_r = fmax(fmax(vl + cl, vr + cr), T(0));
    T ul[5], ur[5], fl[5], fr[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      ul[v] = L.row(l0 + 8 + v);
      ur[v] = R.row(r0 + 8 + v);
      if constexpr (DEV) ur[v] += T(wr[v] - wl[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      fl[v] = L.row(l0 + 16 + v);
      fr[v] = R.row(r0 + 16 + v);
    }
    hll_combine<T, 5>(lam_l, lam_r, ul, fl, ur, fr, out);
    T el[4], er[4], gl[4], gr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      gl[q] = L.row(l0 + mhd_fe_slot(q));
      gr[q] = R.row(r0 + mhd_fe_slot(q));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = mhd_edge_comp(AXIS, q);
      el[q] = L.row(l0 + mhd_ue_slot(q, c));
      er[q] = R.row(r0 + mhd_ue_slot(q, c));
      if constexpr (DEV) er[q] += T(wr[c] - wl[c]);
    }
    hll_combine<T, 4>(lam_l, lam_r, el, gl, er, gr, eout);
    if constexpr (DEV) {
      double Fl[8], Fr[8], Fa[8];
      Mhd<double>::template flux<AXIS>(wl, Fl, gam);
      Mhd<double>::template flux<AXIS>(wr, Fr, gam);
      const double ll = lam_l, lr = lam_r, inv = 1.0 / (lr - ll);
#pragma unroll
      for (int v = 0; v < 8; ++v) Fa[v] = (lr * Fl[v] - ll * Fr[v]) * inv;
#pragma unroll
      for (int v = 0; v < 5; ++v) rf.row(AXIS * 5 + v) = Fa[v] + double(out[v]);
#pragma unroll
      for (int q = 0; q < 4; ++q) re.row(AXIS * 4 + q) = Fa[mhd_edge_comp(AXIS, q)] + double(eout[q]);
      return;
    }
  } else {
    const MhdEigen<T, AXIS> eg(ubl, ubr, tg);
    T du[8], D[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const T a = L.row(l0 + 8 + v);
      du[v] = R.row(r0 + 8 + v) - a;
      if constexpr (DEV) du[v] += T(wr[v] - wl[v]);
    }
    eg.apply(du, D);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T a = L.row(l0 + 16 + v);
      out[v] = T(0.5) * (a + R.row(r0 + 16 + v)) - T(0.5) * D[v];
    }
    T gsum[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T a = L.row(l0 + mhd_fe_slot(q));
      gsum[q] = a + R.row(r0 + mhd_fe_slot(q));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = mhd_edge_comp(AXIS, q);
      T de[8], De[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const T a = L.row(l0 + mhd_ue_slot(q, v));
        de[v] = R.row(r0 + mhd_ue_slot(q, v)) - a;
        if constexpr (DEV) de[v] += T(wr[v] - wl[v]);
      }
      eg.apply(de, De);
      eout[q] = T(0.5) * gsum[q] - T(0.5) * De[c];
    }
    if constexpr (DEV) {
      double Fl[8], Fr[8];
      Mhd<double>::template flux<AXIS>(wl, Fl, gam);
      Mhd<double>::template flux<AXIS>(wr, Fr, gam);
#pragma unroll
      for (int v = 0; v < 5; ++v) rf.row(AXIS * 5 + v) = 0.5 * (Fl[v] + Fr[v]) + double(out[v]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = mhd_edge_comp(AXIS, q);
        re.row(AXIS * 4 + q) = 0.5 * (Fl[c] + Fr[c]) + double(eout[q]);
      }
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) rf.row(AXIS * 5 + v) = double(out[v]);
#pragma unroll
  for (int q = 0; q < 4; ++q) re.row(AXIS * 4 + q) = double(eout[q]);
}

template <class T, int RS, bool DEV>
__host__ __device__ __forceinline__ void face_flux_zone_mhd(const double* __restrict__ U,
                                                            const double* __restrict__ B0,
                                                            const T* __restrict__ PK,
                                                            double* __restrict__ F,
                                                            double* __restrict__ FE, const Grid& g,
                                                            double gam, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  face_flux_axis_mhd<T, RS, 0, DEV>(U, B0, PK, F, FE, g, n, zone_of(wrap(i - 1, g.nx), j, k, g), gam);
  face_flux_axis_mhd<T, RS, 1, DEV>(U, B0, PK, F, FE, g, n, zone_of(i, wrap(j - 1, g.ny), k, g), gam);
  face_flux_axis_mhd<T, RS, 2, DEV>(U, B0, PK, F, FE, g, n, zone_of(i, j, wrap(k - 1, g.nz), g), gam);
}

// Edge fields at the three lower edges of zone n: E_c is the mean of the
// four face values -eps_{dac} Flux_d(B_a) of eq. (7) on the faces that abut
// the edge (edge q = 2 w + (side > 0) of a face, w the transverse slot of a).
__host__ __device__ __forceinline__ void edge_e_zone(const double* __restrict__ FE, double* __restrict__ E,
                                                     const Grid& g, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long mx = zone_of(wrap(i - 1, g.nx), j, k, g);
  const long long my = zone_of(i, wrap(j - 1, g.ny), k, g);
  const long long mz = zone_of(i, j, wrap(k - 1, g.nz), g);
  auto fe = [&](int face, int q, long long zone) { return FE[((long long)face * 4 + q) * g.S + zone]; };
  // E_x: y-faces (component B_z, sign -1), z-faces (component B_y, sign +1)
  double ex = 0.0;
  ex = ex - (fe(1, 2, n) + fe(1, 3, mz));
  ex = ex + (fe(2, 2, n) + fe(2, 3, my));
  // E_y: x-faces (component B_z, sign +1), z-faces (component B_x, sign -1)
  double ey = 0.0;
  ey = ey + (fe(0, 2, n) + fe(0, 3, mz));
  ey = ey - (fe(2, 0, n) + fe(2, 1, mx));
  // E_z: x-faces (component B_y, sign -1), y-faces (component B_x, sign +1)
  double ez = 0.0;
  ez = ez - (fe(0, 0, n) + fe(0, 1, my));
  ez = ez + (fe(1, 0, n) + fe(1, 1, mx));
  E[n] = 0.25 * ex;
  E[g.S + n] = 0.25 * ey;
  E[2 * g.S + n] = 0.25 * ez;
}

// eq. (8) for the three lower faces of zone n (double), with the eq. (6)
// hydro update done by update_zone.
__host__ __device__ __forceinline__ void ct_zone(double* __restrict__ B, const double* __restrict__ E,
                                                 const Grid& g, double h, double dx, double dy,
                                                 double dz, long long n) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long px = zone_of(wrap(i + 1, g.nx), j, k, g);
  const long long py = zone_of(i, wrap(j + 1, g.ny), k, g);
  const long long pz = zone_of(i, j, wrap(k + 1, g.nz), g);
  const double* Ex = E;
  const double* Ey = E + g.S;
  const double* Ez = E + 2 * g.S;
  B[n] = B[n] - h * ((Ez[py] - Ez[n]) / dy - (Ey[pz] - Ey[n]) / dz);
  B[g.S + n] = B[g.S + n] - h * ((Ex[pz] - Ex[n]) / dz - (Ez[px] - Ez[n]) / dx);
  B[2 * g.S + n] = B[2 * g.S + n] - h * ((Ey[px] - Ey[n]) / dx - (Ex[py] - Ex[n]) / dy);
}

// CFL rate of one MHD zone, with the zone field taken as the mean of its
// two face values per component.
__host__ __device__ __forceinline__ double dt_rate_zone_mhd(const double* __restrict__ U,
                                                            const double* __restrict__ B,
                                                            const Grid& g, double gam, double dx,
                                                            double dy, double dz, long long n,
                                                            int& isbad) {
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  double u[8];
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = U[(long long)v * g.S + n];
  u[5] = 0.5 * (B[n] + B[zone_of(wrap(i + 1, g.nx), j, k, g)]);
  u[6] = 0.5 * (B[g.S + n] + B[g.S + zone_of(i, wrap(j + 1, g.ny), k, g)]);
  u[7] = 0.5 * (B[2 * g.S + n] + B[2 * g.S + zone_of(i, j, wrap(k + 1, g.nz), g)]);
  const double p = Mhd<double>::pressure(u, gam);
  bool ok = u[0] > 0.0 && p > 0.0;
#pragma unroll
  for (int v = 0; v < 8; ++v) ok = ok && __builtin_isfinite(u[v]);
  if (!ok) {
    isbad = 1;
    return 0.0;
  }
  return (fabs(u[1] / u[0]) + Mhd<double>::fast_speed<0>(u, gam)) / dx +
         (fabs(u[2] / u[0]) + Mhd<double>::fast_speed<1>(u, gam)) / dy +
         (fabs(u[3] / u[0]) + Mhd<double>::fast_speed<2>(u, gam)) / dz;
}

}  // namespace ader
