// Lane-split layout of the predictor (device only): the NV variables of a
// zone live in NV lanes of one wavefront, one variable per lane, so a lane
// keeps only its own variable's spatial modes, evolutionary modes and
// accumulators (about 65 values at order 4 instead of 65 NV).  Lane
// var * Z + z holds variable var of zone slot z; a wave serves Z = 64 / NV
// zones.  Wherever the scheme needs a whole state (a flux, a positivity
// check) the zone's lanes gather it with ds_bpermute and evaluate it
// redundantly, each keeping its own component.  The generated per-zone code
// runs unchanged with one variable per lane: the flux evaluator and the
// positivity scan below do the gathering.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "zone_ops.h"

namespace ader {

struct SplitLane {
  int var;  // the variable this lane holds
  int z;    // zone slot in the wave
  int Z;    // zones per wave
};

__device__ __forceinline__ float lane_read(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(x)));
}

__device__ __forceinline__ double lane_read(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(lane << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(lane << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// full[c] = variable c of this lane's zone
template <int NV, class T>
__device__ __forceinline__ void gather(const SplitLane& L, T own, T (&full)[NV]) {
#pragma unroll
  for (int c = 0; c < NV; ++c) full[c] = lane_read(own, c * L.Z + L.z);
}

// this lane's component of a full vector (selects, no dynamic indexing)
template <int NV, class T>
__device__ __forceinline__ T pick(const SplitLane& L, const T (&full)[NV]) {
  T r = full[0];
#pragma unroll
  for (int c = 1; c < NV; ++c) r = L.var == c ? full[c] : r;
  return r;
}

// Flux evaluator of the lane-split layout: gathers the zone's state at the
// point, evaluates the whole flux (point or deviation form) and returns this
// lane's component.
template <class P, class T, bool DEV>
struct SplitFlux {
  static constexpr bool kDeviation = DEV;
  static constexpr int comp(int) { return 0; }
  typename FluxOf<P, T, DEV>::type inner;
  SplitLane L;
  template <int AXIS>
  __device__ inline void flux(const T (&u)[1], T (&f)[1]) const {
    T full[P::NV], fl[P::NV];
    gather(L, u[0], full);
    inner.template flux<AXIS>(full, fl);
    f[0] = pick(L, fl);
  }
};

// Positivity scan of the lane-split layout (every lane of a zone scans the
// same gathered states, so the flag agrees across them).
template <class T, int NV, bool DEV>
struct SplitScan {
  static constexpr bool kDeviation = DEV;
  PosScan<T, NV, DEV> inner;
  SplitLane L;
  __device__ void operator()(const T (&u)[1]) {
    T full[NV];
    gather(L, u[0], full);
    inner(full);
  }
};

// Affine source of the lane-split layout: gathers the zone's state at a
// node, forms the whole dt S (point or deviation form) and returns this
// lane's component; base is this lane's component of dt S(zone average),
// which the deviation form's constant source mode takes.
template <class T, bool DEV>
struct SplitSrc {
  static constexpr bool kActive = true;
  AffineSrc<T, DEV> inner;
  SplitLane L;
  T base[1];
  __device__ SplitSrc(const SourceAffine& s, double dt, const double (&w0)[5], const SplitLane& l)
      : inner(s, dt, w0), L(l) {
    base[0] = pick(L, inner.base);
  }
  __device__ void operator()(const T (&u)[1], T (&out)[1]) const {
    T full[5], o[5];
    gather(L, u[0], full);
    inner(full, o);
    out[0] = pick(L, o);
  }
};

// dt (A mean + b) of this lane's variable from the zone's final modes (the
// means of the five lanes gathered); written to SB row L.var at n.
template <class S, class T>
__device__ __forceinline__ void store_source_average_split(const SplitLane& L,
                                                           const SourceAffine& src, double dt,
                                                           const double (&w0)[5],
                                                           const T (&e)[S::NE][1],
                                                           double* __restrict__ SB, long long N,
                                                           long long n) {
  double own[1];
  S::mean_dev(e, own);
  double m[5];
  gather(L, own[0], m);
  double a = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double r = src.b[v];
#pragma unroll
    for (int k = 0; k < 5; ++k) r += src.A[v * 5 + k] * (w0[k] + m[k]);
    a = L.var == v ? r : a;
  }
  SB[(long long)L.var * N + n] = dt * a;
}

// (NoScan: in this layout the facial check set is scanned on its own before
// the sides are formed, which keeps the register use of the side code low.)

// pos_scales for the lanes of one zone: every lane gets the same theta, and
// only the zone's first lane flags or counts.
__device__ __forceinline__ bool pos_scales_lane(const SplitLane& L, const PosCtl& pc,
                                                double theta) {
  if (!(theta < 1.0)) return false;
  if (L.var == 0) return pos_scales(pc, theta);
  return theta >= 0.0;
}

// Exact positivity pass (rare): this lane's component at each check point in
// double, the zone's state gathered, the same theta in every lane of a zone.
template <int NP, int LS, class T, int NV>
__device__ double theta_spatial_split(const SplitLane& L, const double (&w0)[NV],
                                      const T (&w)[LS][1], const double (&phi)[NP][LS],
                                      double gam, bool limit) {
  PosTheta<T, NV> acc(w0, gam, limit);
  const double own0 = pick(L, w0);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double s = own0;
#pragma unroll
    for (int m = 1; m < LS; ++m) s += phi[p][m] * double(w[m][0]);
    double u[NV];
    gather(L, s, u);
    acc(u);
  }
  return acc.result();
}

template <int NP, int LS, int NE, class T, int NV>
__device__ double theta_facial_split(const SplitLane& L, const double (&w0)[NV],
                                     const T (&w)[LS][1], const T (&e)[NE][1],
                                     const double (&phi)[NP][LS + NE], double gam,
                                     bool limit) {
  PosTheta<T, NV> acc(w0, gam, limit);
  const double own0 = pick(L, w0);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double s = own0;
#pragma unroll
    for (int m = 1; m < LS; ++m) s += phi[p][m] * double(w[m][0]);
#pragma unroll
    for (int m = 0; m < NE; ++m) s += phi[p][LS + m] * double(e[m][0]);
    double u[NV];
    gather(L, s, u);
    acc(u);
  }
  return acc.result();
}

// The same operations as predict_zone (Euler), in the lane-split layout;
// SRC: with the affine source *src, whose dt-scaled space-time average goes
// to SB (rows of 5 doubles).
template <class T, int ORDER, int FORM, bool DEV, bool SRC = false>
__device__ __forceinline__ void predict_zone_split(const SplitLane& L, const double* __restrict__ U,
                                                   const T* __restrict__ W, T* __restrict__ PK,
                                                   const Grid& g, double h, double inv_dx,
                                                   double inv_dy, double inv_dz, double gam,
                                                   PosCtl pc, long long n,
                                                   const SourceAffine* src = nullptr,
                                                   double* __restrict__ SB = nullptr) {
  using S = typename SchemeOf<ORDER, FORM, T, 1>::type;
  constexpr int LS = S::LS, NE = S::NE;
  double w0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) w0[v] = U[(long long)v * g.S + n];
  T w[LS][1];
  w[0][0] = DEV ? T(0) : T(pick(L, w0));
#pragma unroll
  for (int m = 1; m < LS; ++m) w[m][0] = W[((long long)(m - 1) * 5 + L.var) * g.S + n];
  {
    SplitScan<T, 5, DEV> scan{PosScan<T, 5, DEV>(w0), L};
    S::spatial_points(w, scan);
    const double theta =
        scan.inner.near ? theta_spatial_split(L, w0, w, S::spatial_phi, gam, pc.limit) : 1.0;
    if (pos_scales_lane(L, pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m) w[m][0] *= th;
    }
  }
  const SplitFlux<Euler<T>, T, DEV> ph{FluxOf<Euler<T>, T, DEV>::make(w0, gam), L};
  T e[NE][1];
  if constexpr (SRC)
    S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph,
               SplitSrc<T, DEV>(*src, h, w0, L));
  else
    S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
  {
    SplitScan<T, 5, DEV> scan{PosScan<T, 5, DEV>(w0), L};
    S::facial_points(w, e, scan);
    const double theta =
        scan.inner.near ? theta_facial_split(L, w0, w, e, S::facial_phi, gam, pc.limit) : 1.0;
    if (pos_scales_lane(L, pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m) w[m][0] *= th;
#pragma unroll
      for (int m = 0; m < NE; ++m) e[m][0] *= th;
    }
  }
  T* base = PK + (long long)L.var * g.S + n;
  auto side = [&](auto side_c) {
    constexpr int SIDE = decltype(side_c)::value;
    T ub[1], ua[1], fa[1];
    NoScan none;
    S::template side<SIDE>(w, e, ph, none, ub, ua, fa);
    base[(long long)((SIDE * 3 + 0) * 5) * g.S] = ub[0];
    base[(long long)((SIDE * 3 + 1) * 5) * g.S] = ua[0];
    base[(long long)((SIDE * 3 + 2) * 5) * g.S] = fa[0];
  };
  side(std::integral_constant<int, 0>{});
  side(std::integral_constant<int, 1>{});
  side(std::integral_constant<int, 2>{});
  side(std::integral_constant<int, 3>{});
  side(std::integral_constant<int, 4>{});
  side(std::integral_constant<int, 5>{});
  // the source term of eq. (6) from the final (possibly scaled) polynomial
  if constexpr (SRC) store_source_average_split<S, T>(L, *src, h, w0, e, SB, g.S, n);
}

// The same operations as predict_zone_mhd, in the lane-split layout.
template <class T, int ORDER, int FORM, bool DEV>
__device__ __forceinline__ void predict_zone_mhd_split(
    const SplitLane& L, const double* __restrict__ U, const T* __restrict__ W,
    const double* __restrict__ B0, const T* __restrict__ WB, const T* __restrict__ BN,
    T* __restrict__ PK, const Grid& g, double h, double inv_dx, double inv_dy, double inv_dz,
    double gam, PosCtl pc, long long n) {
  using S = typename SchemeOf<ORDER, FORM, T, 1>::type;
  constexpr int LS = S::LS, NE = S::NE;
  double w0[8];
#pragma unroll
  for (int v = 0; v < 5; ++v) w0[v] = U[(long long)v * g.S + n];
#pragma unroll
  for (int c = 0; c < 3; ++c) w0[5 + c] = B0[(long long)c * g.S + n];
  const bool field = L.var >= 5;
  // this lane's modes: hydro from W, field from WB
  const T* src = field ? WB + (long long)(L.var - 5) * g.S + n : W + (long long)L.var * g.S + n;
  const long long stride = (long long)(field ? 3 : 5) * g.S;
  T w[LS][1];
  w[0][0] = DEV ? T(0) : T(pick(L, w0));
#pragma unroll
  for (int m = 1; m < LS; ++m) w[m][0] = src[(long long)(m - 1) * stride];
  // the Sec. III normal moments on the pure-normal slots of each field lane
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 1; a < ORDER; ++a) {
      const int m = spatial_mode(c == 0 ? a : 0, c == 1 ? a : 0, c == 2 ? a : 0);
      if (L.var == 5 + c) w[m][0] = BN[((long long)(a - 1) * 3 + c) * g.S + n];
    }
  {
    SplitScan<T, 8, DEV> scan{PosScan<T, 8, DEV>(w0), L};
    S::spatial_points_all(w, scan);
    const double theta =
        scan.inner.near ? theta_spatial_split(L, w0, w, S::spatial_phi_all, gam, pc.limit) : 1.0;
    if (pos_scales_lane(L, pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m) w[m][0] *= th;
    }
  }
  const SplitFlux<Mhd<T>, T, DEV> ph{FluxOf<Mhd<T>, T, DEV>::make(w0, gam), L};
  T e[NE][1];
  S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
  {
    SplitScan<T, 8, DEV> scan{PosScan<T, 8, DEV>(w0), L};
    S::facial_points_all(w, e, scan);
    const double theta =
        scan.inner.near ? theta_facial_split(L, w0, w, e, S::facial_phi_all, gam, pc.limit)
                        : 1.0;
    if (pos_scales_lane(L, pc, theta)) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m) w[m][0] *= th;
#pragma unroll
      for (int m = 0; m < NE; ++m) e[m][0] *= th;
    }
  }
  auto side = [&](auto side_c) {
    constexpr int SIDE = decltype(side_c)::value;
    constexpr int AX = SIDE / 2;
    constexpr int TA0 = AX == 0 ? 1 : 0, TA1 = AX == 2 ? 1 : 2;   // transverse axes
    T ub[1], ua[1], fa[1], ue[4], fe[4];
    NoScan none;
    S::template side_edges<SIDE>(w, e, ph, none, ub, ua, fa, ue, fe);
    T* base = PK + (long long)SIDE * kMhdSlots * g.S + n;
    base[(long long)L.var * g.S] = ub[0];
    base[(long long)(8 + L.var) * g.S] = ua[0];
    base[(long long)(16 + L.var) * g.S] = fa[0];
    // every lane has its own variable's edge averages; the lane holding the
    // field component along an edge's transverse axis has its flux
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      base[(long long)mhd_ue_slot(q, 0) * g.S + (long long)L.var * g.S] = ue[q];
      if (L.var == 5 + (q < 2 ? TA0 : TA1)) base[(long long)mhd_fe_slot(q) * g.S] = fe[q];
    }
  };
  side(std::integral_constant<int, 0>{});
  side(std::integral_constant<int, 1>{});
  side(std::integral_constant<int, 2>{});
  side(std::integral_constant<int, 3>{});
  side(std::integral_constant<int, 4>{});
  side(std::integral_constant<int, 5>{});
}

// ---------------------------------------------------------------------------
// Pair layout (MHD): two lanes per zone, lane g in {0, 1} of a zone holding
// variables 4g .. 4g+3 (rho, m | E, B), so a lane keeps half of the zone's
// modes and accumulators and a whole state costs one exchange of four
// values with the partner lane; the flux is evaluated twice per point (once
// per lane) where the one-variable split evaluates it eight times.  L.var is
// the lane's group g, and a wave serves Z = 32 zones.
constexpr int kPairVars = 4;

// full = the zone's whole state from this lane's half and its partner's
template <int VPL, class T>
__device__ __forceinline__ void pair_gather(const SplitLane& L, const T (&own)[VPL],
                                            T (&full)[2 * VPL]) {
  const int other = (L.var ^ 1) * L.Z + L.z;
#pragma unroll
  for (int k = 0; k < VPL; ++k) {
    const T o = lane_read(own[k], other);
    full[k] = L.var == 0 ? own[k] : o;
    full[VPL + k] = L.var == 0 ? o : own[k];
  }
}

// this lane's half of a whole vector
template <int VPL, class T>
__device__ __forceinline__ void pair_pick(const SplitLane& L, const T (&full)[2 * VPL],
                                          T (&out)[VPL]) {
#pragma unroll
  for (int k = 0; k < VPL; ++k) out[k] = L.var == 0 ? full[k] : full[VPL + k];
}

template <class P, class T, bool DEV>
struct PairFlux {
  static constexpr bool kDeviation = DEV;
  // variable c sits at index c % 4 of the lane that holds it
  static constexpr int comp(int c) { return c % kPairVars; }
  typename FluxOf<P, T, DEV>::type inner;
  SplitLane L;
  template <int AXIS>
  __device__ inline void flux(const T (&u)[kPairVars], T (&f)[kPairVars]) const {
    T full[2 * kPairVars], fl[2 * kPairVars];
    pair_gather(L, u, full);
    inner.template flux<AXIS>(full, fl);
    pair_pick(L, fl, f);
  }
};

template <class T, bool DEV>
struct PairScan {
  static constexpr bool kDeviation = DEV;
  PosScan<T, 2 * kPairVars, DEV> inner;
  SplitLane L;
  __device__ void operator()(const T (&u)[kPairVars]) {
    T full[2 * kPairVars];
    pair_gather(L, u, full);
    inner(full);
  }
};

// Exact positivity pass (rare) of the pair layout: this lane's half at each
// check point in double, the other half from the partner.
template <int NP, int LS, class T>
__device__ double theta_spatial_pair(const SplitLane& L, const double (&w0)[8],
                                     const T (&w)[LS][kPairVars], const double (&phi)[NP][LS],
                                     double gam, bool limit) {
  PosTheta<T, 8> acc(w0, gam, limit);
  double own0[kPairVars];
  pair_pick(L, w0, own0);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double s[kPairVars];
#pragma unroll
    for (int k = 0; k < kPairVars; ++k) {
      s[k] = own0[k];
#pragma unroll
      for (int m = 1; m < LS; ++m) s[k] += phi[p][m] * double(w[m][k]);
    }
    double u[8];
    pair_gather(L, s, u);
    acc(u);
  }
  return acc.result();
}

template <int NP, int LS, int NE, class T>
__device__ double theta_facial_pair(const SplitLane& L, const double (&w0)[8],
                                    const T (&w)[LS][kPairVars], const T (&e)[NE][kPairVars],
                                    const double (&phi)[NP][LS + NE], double gam,
                                    bool limit) {
  PosTheta<T, 8> acc(w0, gam, limit);
  double own0[kPairVars];
  pair_pick(L, w0, own0);
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    double s[kPairVars];
#pragma unroll
    for (int k = 0; k < kPairVars; ++k) {
      s[k] = own0[k];
#pragma unroll
      for (int m = 1; m < LS; ++m) s[k] += phi[p][m] * double(w[m][k]);
#pragma unroll
      for (int m = 0; m < NE; ++m) s[k] += phi[p][LS + m] * double(e[m][k]);
    }
    double u[8];
    pair_gather(L, s, u);
    acc(u);
  }
  return acc.result();
}

// The fluxes of a side packet at the facial nodes (App. D, with the edge
// averages of eq. 57), in the pair layout, from the scheme's point tables:
// one node per iteration of a loop the compiler does not unroll, so beside
// the modes only that node's state and flux are live.  The side kernel of
// the two-kernel form takes it in FP64 at order 4, where the straight-line
// form keeps many nodes' partial sums live and spills 2.7 KB per lane (this
// loop: 0.2 KB; the kernel 19% faster).  In FP32 the straight-line form does
// not spill and the tables' FP64 coefficients would need a conversion per
// lane and use, so FP32 keeps it.
template <class S, int SIDE, class T, class Phys>
__device__ __forceinline__ void side_node_fluxes(const T (&w)[S::LS][kPairVars],
                                                 const T (&e)[S::NE][kPairVars], const Phys& ph,
                                                 T (&fa)[kPairVars], T (&fe)[4]) {
  constexpr int NF = S::NFACE_NODES, LS = S::LS, NE = S::NE;
  constexpr int AX = SIDE / 2;
  constexpr int C0 = Phys::comp(5 + (AX == 0 ? 1 : 0)), C1 = Phys::comp(5 + (AX == 2 ? 1 : 2));
#pragma unroll
  for (int k = 0; k < kPairVars; ++k) fa[k] = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) fe[q] = T(0);
#pragma unroll 1
  for (int j = 0; j < NF; ++j) {
    const double* wt = S::side_node_w[j];
    if (wt[0] == 0.0 && wt[1] == 0.0 && wt[2] == 0.0 && wt[3] == 0.0 && wt[4] == 0.0) continue;
    const double* phi = S::facial_phi_all[SIDE * (NF + 1) + j];
    T u[kPairVars], fl[kPairVars];
#pragma unroll
    for (int k = 0; k < kPairVars; ++k) u[k] = w[0][k];
#pragma unroll
    for (int m = 1; m < LS; ++m)
#pragma unroll
      for (int k = 0; k < kPairVars; ++k) u[k] += T(phi[m]) * w[m][k];
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
      for (int k = 0; k < kPairVars; ++k) u[k] += T(phi[LS + m]) * e[m][k];
    ph.template flux<AX>(u, fl);
#pragma unroll
    for (int k = 0; k < kPairVars; ++k) fa[k] += T(wt[0]) * fl[k];
    fe[0] += T(wt[1]) * fl[C0];
    fe[1] += T(wt[2]) * fl[C0];
    fe[2] += T(wt[3]) * fl[C1];
    fe[3] += T(wt[4]) * fl[C1];
  }
}

// The same operations as predict_zone_mhd, in the pair layout.  EDGES_ALL:
// every variable's edge averages are stored (linearized flux), else only the
// field component each edge needs.  PHASE 0 does it all; PHASE 1 stops after
// the predictor and its positivity scaling, storing the (scaled)
// evolutionary modes in EM (rows m*8 + v) and the two scaling factors in TH
// (rows 0: spatial, 1: facial); PHASE 2 reloads them and forms the side
// packets, so each of the two kernels holds fewer live values.
template <class T, int ORDER, int FORM, bool DEV, bool EDGES_ALL, int PHASE = 0>
__device__ __forceinline__ void predict_zone_mhd_pair(
    const SplitLane& L, const double* __restrict__ U, const T* __restrict__ W,
    const double* __restrict__ B0, const T* __restrict__ WB, const T* __restrict__ BN,
    T* __restrict__ PK, const Grid& g, double h, double inv_dx, double inv_dy, double inv_dz,
    double gam, PosCtl pc, long long n, T* __restrict__ EM = nullptr,
    double* __restrict__ TH = nullptr) {
  constexpr int VPL = kPairVars;
  using S = typename SchemeOf<ORDER, FORM, T, VPL>::type;
  constexpr int LS = S::LS, NE = S::NE;
  double w0[8];
  {
    RowCursor<const double> ru(U, g.S, n), rb(B0, g.S, n);
#pragma unroll
    for (int v = 0; v < 5; ++v) w0[v] = ru.row(v);
#pragma unroll
    for (int c = 0; c < 3; ++c) w0[5 + c] = rb.row(c);
  }
  const int v0 = L.var * VPL;   // first variable of this lane
  T w[LS][VPL];
  {
    double own0[VPL];
    pair_pick(L, w0, own0);
#pragma unroll
    for (int k = 0; k < VPL; ++k) w[0][k] = DEV ? T(0) : T(own0[k]);
  }
  // this lane's modes: variable v from row (m-1) * 5 + v of W (v < 5) or
  // (m-1) * 3 + v - 5 of WB
#pragma unroll
  for (int k = 0; k < VPL; ++k) {
    const int v = v0 + k;
    const bool field = v >= 5;
    const T* q = field ? WB + (long long)(v - 5) * g.S + n : W + (long long)v * g.S + n;
    const long long stride = (long long)(field ? 3 : 5) * g.S;
#pragma unroll
    for (int m = 1; m < LS; ++m) {
      w[m][k] = *q;
      q = next_row(q, stride);
    }
  }
  // the Sec. III normal moments on the pure-normal slots of the field lane
  if (L.var == 1) {
    RowCursor<const T> rn(BN, g.S, n);
#pragma unroll
    for (int a = 1; a < ORDER; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int m = spatial_mode(c == 0 ? a : 0, c == 1 ? a : 0, c == 2 ? a : 0);
        w[m][1 + c] = rn.row((a - 1) * 3 + c);
      }
  }
  double th_s = 1.0;
  {
    if constexpr (PHASE == 2) {
      th_s = TH[n];
    } else {
      PairScan<T, DEV> scan{PosScan<T, 8, DEV>(w0), L};
      S::spatial_points_all(w, scan);
      th_s = scan.inner.near ? theta_spatial_pair(L, w0, w, S::spatial_phi_all, gam, pc.limit)
                             : 1.0;
      // the factor to apply (1 unless the limit mode scales), also what
      // the side kernel of the two-kernel form reloads
      th_s = pos_scales_lane(L, pc, th_s) ? th_s : 1.0;
    }
    const double theta = th_s;
    if (theta < 1.0) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int k = 0; k < VPL; ++k) w[m][k] *= th;
    }
  }
  const PairFlux<Mhd<T>, T, DEV> ph{FluxOf<Mhd<T>, T, DEV>::make(w0, gam), L};
  T e[NE][VPL];
  if constexpr (PHASE == 2) {
    const double theta = TH[g.S + n];
    if (theta < 1.0) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int k = 0; k < VPL; ++k) w[m][k] *= th;
    }
    RowCursor<const T> re(EM, g.S, n, v0);
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
      for (int k = 0; k < VPL; ++k) e[m][k] = re.row(m * 8 + v0 + k);
  } else {
    S::predict(w, e, T(h * inv_dx), T(h * inv_dy), T(h * inv_dz), ph);
    PairScan<T, DEV> scan{PosScan<T, 8, DEV>(w0), L};
    S::facial_points_all(w, e, scan);
    const double theta_x =
        scan.inner.near ? theta_facial_pair(L, w0, w, e, S::facial_phi_all, gam, pc.limit) : 1.0;
    const double theta = pos_scales_lane(L, pc, theta_x) ? theta_x : 1.0;
    if (theta < 1.0) {
      const T th = T(theta);
#pragma unroll
      for (int m = 1; m < LS; ++m)
#pragma unroll
        for (int k = 0; k < VPL; ++k) w[m][k] *= th;
#pragma unroll
      for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int k = 0; k < VPL; ++k) e[m][k] *= th;
    }
    if constexpr (PHASE == 1) {
      RowCursor<T> re(EM, g.S, n, v0);
#pragma unroll
      for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int k = 0; k < VPL; ++k) re.row(m * 8 + v0 + k) = e[m][k];
      if (L.var == 0) {
        TH[n] = th_s;
        TH[g.S + n] = theta;
      }
      return;
    }
  }
  auto side = [&](auto side_c) {
    constexpr int SIDE = decltype(side_c)::value;
    constexpr int AX = SIDE / 2;
    constexpr int TA0 = AX == 0 ? 1 : 0, TA1 = AX == 2 ? 1 : 2;   // transverse axes
    T ub[VPL], ua[VPL], fa[VPL], ue[4], fe[4];
    if constexpr (PHASE == 2 && ORDER == 4 && std::is_same<T, double>::value) {
      S::template side_linear<SIDE, PairFlux<Mhd<T>, T, DEV>>(w, e, ub, ua, ue);
      side_node_fluxes<S, SIDE>(w, e, ph, fa, fe);
    } else {
      NoScan none;
      S::template side_edges<SIDE>(w, e, ph, none, ub, ua, fa, ue, fe);
    }
    T* base = PK + (long long)SIDE * kMhdSlots * g.S + n;
    RowCursor<T> r(base + (long long)v0 * g.S, g.S, 0);
#pragma unroll
    for (int k = 0; k < VPL; ++k) r.row(k) = ub[k];
#pragma unroll
    for (int k = 0; k < VPL; ++k) r.row(8 + k) = ua[k];
#pragma unroll
    for (int k = 0; k < VPL; ++k) r.row(16 + k) = fa[k];
    if constexpr (EDGES_ALL && PHASE == 2 && ORDER == 4 && std::is_same<T, double>::value) {
      // every variable's edge averages (linearized solver), as the node
      // fluxes above: one edge at a time from the tables (the straight-line
      // form spilled 1 KB per lane here; this loop none, the kernel pair
      // 10% faster)
#pragma unroll 1
      for (int q = 0; q < 4; ++q) {
        const double* row = S::edge_rows_all[SIDE][q];
        T ue_q[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) ue_q[k] = DEV ? T(0) : T(row[0]) * w[0][k];
#pragma unroll
        for (int m = 1; m < LS; ++m)
#pragma unroll
          for (int k = 0; k < VPL; ++k) ue_q[k] += T(row[m]) * w[m][k];
#pragma unroll
        for (int m = 0; m < NE; ++m)
#pragma unroll
          for (int k = 0; k < VPL; ++k) ue_q[k] += T(row[LS + m]) * e[m][k];
#pragma unroll
        for (int k = 0; k < VPL; ++k) r.row(mhd_ue_slot(q, k)) = ue_q[k];
      }
    } else if constexpr (EDGES_ALL) {
      T ues[4][VPL];
      S::template edge_states<SIDE, DEV>(w, e, ues);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < VPL; ++k) r.row(mhd_ue_slot(q, k)) = ues[q][k];
    }
    // the field lane has the field components along the edges' transverse
    // axes: their edge averages (HLL) and their edge fluxes
    if (L.var == 1) {
      RowCursor<T> rf(base, g.S, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) rf.row(mhd_fe_slot(q)) = fe[q];
      if constexpr (!EDGES_ALL) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rf.row(mhd_ue_slot(q, 5 + (q < 2 ? TA0 : TA1))) = ue[q];
      }
    }
  };
  side(std::integral_constant<int, 0>{});
  side(std::integral_constant<int, 1>{});
  side(std::integral_constant<int, 2>{});
  side(std::integral_constant<int, 3>{});
  side(std::integral_constant<int, 4>{});
  side(std::integral_constant<int, 5>{});
}

}  // namespace ader
