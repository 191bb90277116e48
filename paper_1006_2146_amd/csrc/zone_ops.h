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
//   F   T      [3][5][N]         numerical flux at the lower x/y/z face of each
//                                zone (eq. 56 or the linearized flux)
// T is double on the FP64 path and float on the mixed path; U, the update and
// dt stay double on both.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "euler_device.h"
#include "generated/ader_scheme.h"

namespace ader {

struct Grid {
  int nx, ny, nz;
  long long N;
};

__host__ __device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

__host__ __device__ __forceinline__ long long zone_of(int i, int j, int k, const Grid& g) {
  return ((long long)k * g.ny + j) * g.nx + i;
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
    const T a0 = T(1) / (e0 * e0), a1 = T(100) / (e1 * e1), a2 = T(1) / (e2 * e2);
    const T tot = a0 + a1 + a2;
    m[1] = (a0 * c0[1] + a1 * c1[1] + a2 * c2[1]) / tot;
    m[2] = (a0 * c0[2] + a1 * c1[2] + a2 * c2[2]) / tot;
  } else {
    T c[4][4];
    ader_gen::Weno4<T>::cand0(d, c[0]);
    ader_gen::Weno4<T>::cand1(d, c[1]);
    ader_gen::Weno4<T>::cand2(d, c[2]);
    ader_gen::Weno4<T>::cand3(d, c[3]);
    T a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T t = c[s][1] + T(0.1) * c[s][3];
      const T is = t * t + T(13.0 / 3.0) * c[s][2] * c[s][2] + T(781.0 / 20.0) * c[s][3] * c[s][3];
      const T e = T(kEps) + is;
      a[s] = ((s == 1 || s == 2) ? T(100) : T(1)) / (e * e);
    }
    const T tot = a[0] + a[1] + a[2] + a[3];
#pragma unroll
    for (int q = 1; q < 4; ++q)
      m[q] = (a[0] * c[0][q] + a[1] * c[1][q] + a[2] * c[2][q] + a[3] * c[3][q]) / tot;
  }
}

// One sweep of the dimension-by-dimension reconstruction along AXIS.
// x: the zone averages give the x-moments (a,0,0);  y: each field (a,0,0),
// a <= M-2, gives (a,b,0);  z: each field (a,b,0), a+b <= M-2, gives (a,b,c);
// moments of total degree > M-1 are not formed.
template <class T, int M, int AXIS>
__host__ __device__ __forceinline__ void weno_sweep_zone(const double* __restrict__ U,
                                                         T* __restrict__ W, const Grid& g,
                                                         long long n) {
  const int i = (int)(n % g.nx);
  const int j = (int)((n / g.nx) % g.ny);
  const int k = (int)(n / ((long long)g.nx * g.ny));
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
      for (int v = 0; v < 5; ++v) {
        T d[2 * M - 1];
#pragma unroll
        for (int q = 0; q < 2 * R + 1; ++q)
          d[q] = src == 0 ? T(U[(long long)v * g.N + idx[q]])
                          : W[((long long)(src - 1) * 5 + v) * g.N + idx[q]];
        T mo[M];
        weno1d<T, M>(d, mo);
#pragma unroll
        for (int c = 1; c <= M - 1; ++c) {
          if (c > nout) continue;
          int dst;
          if constexpr (AXIS == 0) dst = spatial_mode(c, 0, 0);
          else if constexpr (AXIS == 1) dst = spatial_mode(a, c, 0);
          else dst = spatial_mode(a, b, c);
          W[((long long)(dst - 1) * 5 + v) * g.N + n] = mo[c];
        }
      }
    }
  }
}

// Second order: per axis the minmod of the two one-sided differences
// (the limiter of the second-order workload).
template <class T>
__host__ __device__ __forceinline__ void minmod_zone(const double* __restrict__ U,
                                                     T* __restrict__ W, const Grid& g,
                                                     long long n) {
  const int i = (int)(n % g.nx);
  const int j = (int)((n / g.nx) % g.ny);
  const int k = (int)(n / ((long long)g.nx * g.ny));
  const long long nb[3][2] = {
      {zone_of(wrap(i - 1, g.nx), j, k, g), zone_of(wrap(i + 1, g.nx), j, k, g)},
      {zone_of(i, wrap(j - 1, g.ny), k, g), zone_of(i, wrap(j + 1, g.ny), k, g)},
      {zone_of(i, j, wrap(k - 1, g.nz), g), zone_of(i, j, wrap(k + 1, g.nz), g)}};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double c = U[(long long)v * g.N + n];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double fwd = U[(long long)v * g.N + nb[ax][1]] - c;
      const double bwd = c - U[(long long)v * g.N + nb[ax][0]];
      double s = 0.0;
      if (fwd * bwd > 0.0) s = fabs(fwd) < fabs(bwd) ? fwd : bwd;
      W[((long long)ax * 5 + v) * g.N + n] = T(s);
    }
  }
}

// ---------------------------------------------------------------------------
// Positivity safeguard (the reading that keeps strong blasts physical: one
// Zhang-Shu scaling factor per zone polynomial, computed in double).
// ---------------------------------------------------------------------------
template <class T>
struct PosTheta {
  double ub[5];
  double eps_rho, eps_p, gam, theta;

  __host__ __device__ PosTheta(const T (&w0)[5], double g) : gam(g), theta(1.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) ub[v] = double(w0[v]);
    eps_rho = 1.0e-8 * ub[0];
    const double pb = (gam - 1.0) * (ub[4] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]) / ub[0]);
    eps_p = 1.0e-8 * pb;
  }

  // smallest t in (0, 1] where the pressure along ub + t (u - ub) falls to
  // eps_p: root of rho(t)(E(t) - e) - |m(t)|^2/2 = a t^2 + b t + c
  __host__ __device__ double pressure_root(const double (&du)[5]) const {
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

  // theta = min over points of the largest admissible scale along the line
  // from the zone average to the point: the density bound (linear) and the
  // first crossing of the pressure bound (root above); the same value as
  // scaling for density first and then for pressure.
  __host__ __device__ void operator()(const T (&uT)[5]) {
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = double(uT[v]);
    const double p = (gam - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
    if (u[0] < eps_rho || p < eps_p) {
      double t = 1.0;
      if (u[0] < eps_rho) t = (ub[0] - eps_rho) / (ub[0] - u[0]);
      double du[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) du[v] = u[v] - ub[v];
      t = fmin(t, pressure_root(du));
      theta = fmin(theta, t);
    }
  }
};

// Cheap scan of the same points: flags a zone whose polynomial comes near
// the bounds (within a factor 2, so that rounding in T never hides a
// violation); only such zones run the exact pass in double.
template <class T>
struct PosScan {
  T eps_rho, eps_e;
  int near = 0;
  __host__ __device__ PosScan(const T (&w0)[5], T gam) {
    // internal energy per volume of the zone average, and twice-relaxed bounds
    const T rhoe = w0[4] - T(0.5) * (w0[1] * w0[1] + w0[2] * w0[2] + w0[3] * w0[3]) / w0[0];
    eps_rho = T(2.0e-8) * w0[0];
    eps_e = T(2.0e-8) * rhoe;
    (void)gam;
  }
  // rho >= eps_rho and rho E - |m|^2/2 >= rho eps_e, free of divisions
  __host__ __device__ void operator()(const T (&u)[5]) {
    const T m2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const int ok = int(u[0] >= eps_rho) & int(u[0] * u[4] - T(0.5) * m2 >= u[0] * eps_e);
    near |= ok ^ 1;
  }
};

// Exact pass for a flagged zone: a runtime loop over the check points with
// the basis values from the scheme's tables, so the rare path stays small.
template <class S, class T>
__host__ __device__ double theta_spatial(const T (&w)[S::LS][5], double gam) {
  PosTheta<T> acc(w[0], gam);
#pragma unroll 1
  for (int p = 0; p < S::NSPATIAL; ++p) {
    T u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T s = T(0);
#pragma unroll
      for (int m = 0; m < S::LS; ++m) s += T(S::spatial_phi[p][m]) * w[m][v];
      u[v] = s;
    }
    acc(u);
  }
  return acc.theta;
}

template <class S, class T>
__host__ __device__ double theta_facial(const T (&w)[S::LS][5], const T (&e)[S::NE][5], double gam) {
  PosTheta<T> acc(w[0], gam);
#pragma unroll 1
  for (int p = 0; p < S::NFACIAL; ++p) {
    T u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T s = T(0);
#pragma unroll
      for (int m = 0; m < S::LS; ++m) s += T(S::facial_phi[p][m]) * w[m][v];
#pragma unroll
      for (int m = 0; m < S::NE; ++m) s += T(S::facial_phi[p][S::LS + m]) * e[m][v];
      u[v] = s;
    }
    acc(u);
  }
  return acc.theta;
}

template <int ORDER, int FORM, class T>
struct SchemeOf;
template <class T> struct SchemeOf<2, 0, T> { using type = ader_gen::SchemeM2<T, 5>; };
template <class T> struct SchemeOf<2, 1, T> { using type = ader_gen::SchemeN2<T, 5>; };
template <class T> struct SchemeOf<3, 0, T> { using type = ader_gen::SchemeM3<T, 5>; };
template <class T> struct SchemeOf<4, 0, T> { using type = ader_gen::SchemeM4<T, 5>; };

template <class S, class T, int SIDE>
__host__ __device__ __forceinline__ void store_side(const T (&w)[S::LS][5], const T (&e)[S::NE][5], T gam,
                                           T* __restrict__ PK, long long N, long long n) {
  T ub[5], ua[5], fa[5];
  S::template side<SIDE, Euler<T>>(w, e, gam, ub, ua, fa);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    PK[((long long)(SIDE * 3 + 0) * 5 + v) * N + n] = ub[v];
    PK[((long long)(SIDE * 3 + 1) * 5 + v) * N + n] = ua[v];
    PK[((long long)(SIDE * 3 + 2) * 5 + v) * N + n] = fa[v];
  }
}

// Per zone: load the reconstruction, positivity scaling, space-time predictor
// (Sec. IV / App. A), positivity scaling, and the six face-side packets.
template <class T, int ORDER, int FORM>
__host__ __device__ __forceinline__ void predict_zone(const double* __restrict__ U,
                                                      const T* __restrict__ W,
                                                      T* __restrict__ PK, const Grid& g,
                                                      double h, double inv_dx, double inv_dy,
                                                      double inv_dz, double gam, long long n) {
  using S = typename SchemeOf<ORDER, FORM, T>::type;
  constexpr int LS = S::LS, NE = S::NE;
  T w[LS][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[0][v] = T(U[(long long)v * g.N + n]);
#pragma unroll
  for (int m = 1; m < LS; ++m)
#pragma unroll
    for (int v = 0; v < 5; ++v) w[m][v] = W[((long long)(m - 1) * 5 + v) * g.N + n];

  {
    PosScan<T> scan(w[0], T(gam));
    S::spatial_points(w, scan);
    const double theta = scan.near ? theta_spatial<S, T>(w, gam) : 1.0;
    if (theta < 1.0) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w[m][v] *= th;
    }
  }
  T e[NE][5];
  S::template predict<Euler<T>>(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), T(gam));
  {
    PosScan<T> scan(w[0], T(gam));
    S::facial_points(w, e, scan);
    const double theta = scan.near ? theta_facial<S, T>(w, e, gam) : 1.0;
    if (theta < 1.0) {
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
  }
  const T tg = T(gam);
  store_side<S, T, 0>(w, e, tg, PK, g.N, n);
  store_side<S, T, 1>(w, e, tg, PK, g.N, n);
  store_side<S, T, 2>(w, e, tg, PK, g.N, n);
  store_side<S, T, 3>(w, e, tg, PK, g.N, n);
  store_side<S, T, 4>(w, e, tg, PK, g.N, n);
  store_side<S, T, 5>(w, e, tg, PK, g.N, n);
}

// ---------------------------------------------------------------------------
// Riemann fluxes at the faces (Sec. II.3, V): wave structure frozen at the
// two barycentre states.
// ---------------------------------------------------------------------------
template <class T, int AXIS>
__host__ __device__ __forceinline__ void hll_flux(const T (&ubl)[5], const T (&ul)[5], const T (&fl)[5],
                                         const T (&ubr)[5], const T (&ur)[5], const T (&fr)[5],
                                         T gam, T (&out)[5]) {
  const T vl = ubl[1 + AXIS] / ubl[0], vr = ubr[1 + AXIS] / ubr[0];
  const T cl = sqrt(gam * Euler<T>::pressure(ubl, gam) / ubl[0]);
  const T cr = sqrt(gam * Euler<T>::pressure(ubr, gam) / ubr[0]);
  const T lam_l = fmin(fmin(vl - cl, vr - cr), T(0));
  const T lam_r = fmax(fmax(vl + cl, vr + cr), T(0));
  const T inv = T(1) / (lam_r - lam_l);
#pragma unroll
  for (int v = 0; v < 5; ++v)
    out[v] = (lam_r * fl[v] - lam_l * fr[v] + lam_r * lam_l * (ur[v] - ul[v])) * inv;
}

// Linearized flux: (F_L + F_R)/2 - R |Lambda| L (u_R - u_L)/2 with the Euler
// eigen-system at the mean of the two barycentre primitive states.
template <class T, int AXIS>
__host__ __device__ __forceinline__ void linearized_flux(const T (&ubl)[5], const T (&ul)[5], const T (&fl)[5],
                                                const T (&ubr)[5], const T (&ur)[5], const T (&fr)[5],
                                                T gam, T (&out)[5]) {
  constexpr int A = 1 + AXIS;
  constexpr int B = AXIS == 0 ? 2 : 1;
  constexpr int C = AXIS == 2 ? 2 : 3;
  const T rl = ubl[0], rr = ubr[0];
  const T pl = Euler<T>::pressure(ubl, gam), pr = Euler<T>::pressure(ubr, gam);
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

template <class T, int RS, int AXIS>
__host__ __device__ __forceinline__ void face_flux_axis(const T* __restrict__ PK, T* __restrict__ F,
                                               const Grid& g, long long n, long long nl, T gam) {
  T ubl[5], ul[5], fl[5], ubr[5], ur[5], fr[5], out[5];
  constexpr int SL = 2 * AXIS + 1, SR = 2 * AXIS;  // top side of the lower zone, bottom side of this
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    ubl[v] = PK[((long long)(SL * 3 + 0) * 5 + v) * g.N + nl];
    ul[v] = PK[((long long)(SL * 3 + 1) * 5 + v) * g.N + nl];
    fl[v] = PK[((long long)(SL * 3 + 2) * 5 + v) * g.N + nl];
    ubr[v] = PK[((long long)(SR * 3 + 0) * 5 + v) * g.N + n];
    ur[v] = PK[((long long)(SR * 3 + 1) * 5 + v) * g.N + n];
    fr[v] = PK[((long long)(SR * 3 + 2) * 5 + v) * g.N + n];
  }
  if constexpr (RS == 0) hll_flux<T, AXIS>(ubl, ul, fl, ubr, ur, fr, gam, out);
  else linearized_flux<T, AXIS>(ubl, ul, fl, ubr, ur, fr, gam, out);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[((long long)AXIS * 5 + v) * g.N + n] = out[v];
}

// Each face flux is formed once, by the zone above it, so both zones that
// share a face see the same value and the update conserves exactly.
template <class T, int RS>
__host__ __device__ __forceinline__ void face_flux_zone(const T* __restrict__ PK, T* __restrict__ F,
                                                        const Grid& g, double gam, long long n) {
  const int i = (int)(n % g.nx);
  const int j = (int)((n / g.nx) % g.ny);
  const int k = (int)(n / ((long long)g.nx * g.ny));
  face_flux_axis<T, RS, 0>(PK, F, g, n, zone_of(wrap(i - 1, g.nx), j, k, g), T(gam));
  face_flux_axis<T, RS, 1>(PK, F, g, n, zone_of(i, wrap(j - 1, g.ny), k, g), T(gam));
  face_flux_axis<T, RS, 2>(PK, F, g, n, zone_of(i, j, wrap(k - 1, g.nz), g), T(gam));
}

// eq. (6) in double: U -= dt/dx (F_{i+1/2} - F_{i-1/2}) + ... (y, z)
template <class T>
__host__ __device__ __forceinline__ void update_zone(double* __restrict__ U, const T* __restrict__ F,
                                                     const Grid& g, double h, double dx,
                                                     double dy, double dz, long long n) {
  const int i = (int)(n % g.nx);
  const int j = (int)((n / g.nx) % g.ny);
  const int k = (int)(n / ((long long)g.nx * g.ny));
  const long long up[3] = {zone_of(wrap(i + 1, g.nx), j, k, g), zone_of(i, wrap(j + 1, g.ny), k, g),
                           zone_of(i, j, wrap(k + 1, g.nz), g)};
  const double c[3] = {h / dx, h / dy, h / dz};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double u = U[(long long)v * g.N + n];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double fp = double(F[((long long)ax * 5 + v) * g.N + up[ax]]);
      const double fm = double(F[((long long)ax * 5 + v) * g.N + n]);
      u = u - c[ax] * (fp - fm);
    }
    U[(long long)v * g.N + n] = u;
  }
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
  const double m[3] = {U[g.N + n], U[2 * g.N + n], U[3 * g.N + n]};
  const double E = U[4 * g.N + n];
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

}  // namespace ader
