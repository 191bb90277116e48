// Host build of the HIP kernel source, for CPU tests only.
//
// Runs the same per-zone functions the GPU kernels call (zone_ops.h),
// zone by zone in stage order on the CPU, so the CPU test suite can check the
// kernel logic (generated scheme code, WENO sweeps, positivity scaling,
// Riemann fluxes, update) against the oracle before any GPU run.  It is not
// part of the library and nothing in the product path loads it.
#include <cstdlib>
#include <vector>

#include "../../paper_1006_2146_amd/csrc/zone_ops.h"

using namespace ader;

// Positivity handling of the host build: the mode set by
// hostemu_set_positivity, and the problem's flag and scaling count.
static int g_limit = 0, g_bad = 0;
static unsigned int g_limited = 0;
static PosCtl emu_pc() { return PosCtl{g_limit, &g_bad, &g_limited}; }

// The affine source term of the host build (hostemu_set_source).
static bool g_has_src = false;
static SourceAffine g_src{};

template <class T, int ORDER, int FORM, bool DEV>
static void emu_predict(const double* U, const T* W, T* PK, double* SB, const Grid& g, double dt,
                        double ix, double iy, double iz, double gam, long long n) {
  if (g_has_src)
    predict_zone<T, ORDER, FORM, DEV, true, true>(U, W, PK, g, dt, ix, iy, iz, gam, emu_pc(), n,
                                                  &g_src, SB);
  else
    predict_zone<T, ORDER, FORM, DEV>(U, W, PK, g, dt, ix, iy, iz, gam, emu_pc(), n);
}

template <class T, bool DEV>
static void emu_step(double* U, Grid g, double dx, double dy, double dz, double gam, int order,
                     int form, int riemann, double dt) {
  std::vector<T> W((size_t)19 * 5 * g.N), PK((size_t)90 * g.N);
  std::vector<double> F((size_t)15 * g.N), SB(g_has_src ? (size_t)5 * g.N : 0);
  const long long N = g.N;
  if (order == 2) {
    for (long long n = 0; n < N; ++n) minmod_zone<T>(U, W.data(), g, n);
  } else if (order == 3) {
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 0>(U, W.data(), g, n);
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 1>(U, W.data(), g, n);
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 2>(U, W.data(), g, n);
  } else {
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 0>(U, W.data(), g, n);
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 1>(U, W.data(), g, n);
    for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 2>(U, W.data(), g, n);
  }
  const double ix = 1.0 / dx, iy = 1.0 / dy, iz = 1.0 / dz;
  for (long long n = 0; n < N; ++n) {
    const T* w = W.data();
    T* pk = PK.data();
    double* sb = SB.data();
    if (order == 2 && form == 1)
      emu_predict<T, 2, 1, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
    else if (order == 2)
      emu_predict<T, 2, 0, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
    else if (order == 3 && form == 1)
      emu_predict<T, 3, 1, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
    else if (order == 4 && form == 1)
      emu_predict<T, 4, 1, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
    else if (order == 3)
      emu_predict<T, 3, 0, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
    else
      emu_predict<T, 4, 0, DEV>(U, w, pk, sb, g, dt, ix, iy, iz, gam, n);
  }
  for (long long n = 0; n < N; ++n) {
    if (riemann == 0)
      face_flux_zone<T, 0, DEV>(U, PK.data(), F.data(), g, gam, n);
    else
      face_flux_zone<T, 1, DEV>(U, PK.data(), F.data(), g, gam, n);
  }
  for (long long n = 0; n < N; ++n) {
    update_zone(U, F.data(), g, dt, dx, dy, dz, n);
    if (g_has_src) source_zone(U, SB.data(), g, n);
  }
}

// One SSP-RK step (Sec. II.d) of the Euler equations from the RK kernels'
// per-zone functions: the stage weights of eq. (18), (19) and (20) are
// restated here (the host build has no access to the library's table).
template <class T, bool DEV>
static void emu_rk_step(double* U, Grid g, double dx, double dy, double dz, double gam,
                        int order, int riemann, double dt) {
  struct Row { double a_n, a_c, c_l, a_2, a_3, c_d; int keep; };
  static const Row rk2[] = {{0, 1, 1, 0, 0, 0, 0}, {0.5, 0.5, 0.5, 0, 0, 0, 0}};
  static const Row rk3[] = {{0, 1, 1, 0, 0, 0, 0}, {0.75, 0.25, 0.25, 0, 0, 0, 0},
                            {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 0, 0, 0, 0}};
  static const Row rk54[] = {
      {0, 1, 0.39175222700392, 0, 0, 0, 0},
      {0.44437049406734, 0.55562950593266, 0.36841059262959, 0, 0, 0, 2},
      {0.62010185138540, 0.37989814861460, 0.25189177424738, 0, 0, 0, 3},
      {0.17807995410773, 0.82192004589227, 0.54497475021237, 0, 0, 0, 4},
      {0.00683325884039, 0.34833675773694, 0.22600748319395, 0.51723167208978,
       0.12759831133288, 0.08460416338212, 0}};
  const Row* rows = order == 2 ? rk2 : order == 3 ? rk3 : rk54;
  const int nst = order == 2 ? 2 : order == 3 ? 3 : 5;
  const long long N = g.N;
  std::vector<T> W((size_t)19 * 5 * N), PK((size_t)90 * N);
  std::vector<double> F((size_t)15 * N), Un(U, U + 5 * N), S2(5 * N), S3(5 * N), D3(5 * N);
  for (int s = 0; s < nst; ++s) {
    if (order == 2) {
      for (long long n = 0; n < N; ++n) minmod_zone<T>(U, W.data(), g, n);
    } else if (order == 3) {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 0>(U, W.data(), g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 1>(U, W.data(), g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 2>(U, W.data(), g, n);
    } else {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 0>(U, W.data(), g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 1>(U, W.data(), g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 2>(U, W.data(), g, n);
    }
    for (long long n = 0; n < N; ++n) {
      if (order == 2) rk_sides_zone<T, 2, DEV>(U, W.data(), PK.data(), g, gam, emu_pc(), n);
      else if (order == 3) rk_sides_zone<T, 3, DEV>(U, W.data(), PK.data(), g, gam, emu_pc(), n);
      else rk_sides_zone<T, 4, DEV>(U, W.data(), PK.data(), g, gam, emu_pc(), n);
    }
    for (long long n = 0; n < N; ++n) {
      if (riemann == 0) face_flux_zone<T, 0, DEV>(U, PK.data(), F.data(), g, gam, n);
      else face_flux_zone<T, 1, DEV>(U, PK.data(), F.data(), g, gam, n);
    }
    const Row& r = rows[s];
    const RkStage st{r.a_n, r.a_c, r.c_l, r.a_2, r.a_3, r.c_d, Un.data(), S2.data(), S3.data(),
                     D3.data(), r.keep == 2 ? S2.data() : r.keep == 3 ? S3.data() : nullptr,
                     r.keep == 4 ? D3.data() : nullptr};
    for (long long n = 0; n < N; ++n) rk_stage_zone(U, F.data(), st, g, dt, dx, dy, dz, n);
  }
}

template <class T>
static void emu_recon(const double* src, T* W, Grid g, int order, int nvar) {
  const long long N = g.N;
  if (nvar == 5) {
    if (order == 2) for (long long n = 0; n < N; ++n) minmod_zone<T, 5>(src, W, g, n);
    if (order == 3) {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 0, 5>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 1, 5>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 2, 5>(src, W, g, n);
    }
    if (order == 4) {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 0, 5>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 1, 5>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 2, 5>(src, W, g, n);
    }
  } else {
    if (order == 2) for (long long n = 0; n < N; ++n) minmod_zone<T, 3>(src, W, g, n);
    if (order == 3) {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 0, 3>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 1, 3>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 3, 2, 3>(src, W, g, n);
    }
    if (order == 4) {
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 0, 3>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 1, 3>(src, W, g, n);
      for (long long n = 0; n < N; ++n) weno_sweep_zone<T, 4, 2, 3>(src, W, g, n);
    }
  }
}

template <class T, bool DEV, int RS>
static void emu_step_mhd(double* U, double* B, Grid g, double dx, double dy, double dz, double gam,
                         int order, int form, double dt) {
  constexpr bool ALL = RS == 1;
  const long long N = g.N;
  std::vector<T> W((size_t)19 * 5 * N), WB((size_t)19 * 3 * N), BN((size_t)9 * N),
      PK((size_t)6 * kMhdSlots * N);
  std::vector<double> B0((size_t)3 * N), E((size_t)3 * N), F((size_t)15 * N), FE((size_t)12 * N);
  for (long long n = 0; n < N; ++n) {
    if (order == 2) bface_zone<T, 2>(B, B0.data(), BN.data(), g, n);
    if (order == 3) bface_zone<T, 3>(B, B0.data(), BN.data(), g, n);
    if (order == 4) bface_zone<T, 4>(B, B0.data(), BN.data(), g, n);
  }
  emu_recon<T>(U, W.data(), g, order, 5);
  emu_recon<T>(B0.data(), WB.data(), g, order, 3);
  const double ix = 1.0 / dx, iy = 1.0 / dy, iz = 1.0 / dz;
  for (long long n = 0; n < N; ++n) {
    if (order == 2 && form == 1)
      predict_zone_mhd<T, 2, 1, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
    else if (order == 2)
      predict_zone_mhd<T, 2, 0, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
    else if (order == 3 && form == 1)
      predict_zone_mhd<T, 3, 1, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
    else if (order == 4 && form == 1)
      predict_zone_mhd<T, 4, 1, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
    else if (order == 3)
      predict_zone_mhd<T, 3, 0, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
    else
      predict_zone_mhd<T, 4, 0, DEV, true, ALL>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, dt, ix, iy, iz, gam, emu_pc(), n);
  }
  for (long long n = 0; n < N; ++n)
    face_flux_zone_mhd<T, RS, DEV>(U, B0.data(), PK.data(), F.data(), FE.data(), g, gam, n);
  for (long long n = 0; n < N; ++n) edge_e_zone(FE.data(), E.data(), g, n);
  for (long long n = 0; n < N; ++n) update_zone(U, F.data(), g, dt, dx, dy, dz, n);
  for (long long n = 0; n < N; ++n) ct_zone(B, E.data(), g, dt, dx, dy, dz, n);
}

// One SSP-RK step of ideal MHD from the RK kernels' per-zone functions
// (stage weights of eq. 18-20 restated as in emu_rk_step).
template <class T, bool DEV, int RS>
static void emu_rk_step_mhd(double* U, double* B, Grid g, double dx, double dy, double dz,
                            double gam, int order, double dt) {
  constexpr bool ALL = RS == 1;
  struct Row { double a_n, a_c, c_l, a_2, a_3, c_d; int keep; };
  static const Row rk2[] = {{0, 1, 1, 0, 0, 0, 0}, {0.5, 0.5, 0.5, 0, 0, 0, 0}};
  static const Row rk3[] = {{0, 1, 1, 0, 0, 0, 0}, {0.75, 0.25, 0.25, 0, 0, 0, 0},
                            {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 0, 0, 0, 0}};
  static const Row rk54[] = {
      {0, 1, 0.39175222700392, 0, 0, 0, 0},
      {0.44437049406734, 0.55562950593266, 0.36841059262959, 0, 0, 0, 2},
      {0.62010185138540, 0.37989814861460, 0.25189177424738, 0, 0, 0, 3},
      {0.17807995410773, 0.82192004589227, 0.54497475021237, 0, 0, 0, 4},
      {0.00683325884039, 0.34833675773694, 0.22600748319395, 0.51723167208978,
       0.12759831133288, 0.08460416338212, 0}};
  const Row* rows = order == 2 ? rk2 : order == 3 ? rk3 : rk54;
  const int nst = order == 2 ? 2 : order == 3 ? 3 : 5;
  const long long N = g.N;
  std::vector<T> W((size_t)19 * 5 * N), WB((size_t)19 * 3 * N), BN((size_t)9 * N),
      PK((size_t)6 * kMhdSlots * N);
  std::vector<double> B0((size_t)3 * N), E((size_t)3 * N), F((size_t)15 * N), FE((size_t)12 * N);
  std::vector<double> Un(U, U + 5 * N), S2(5 * N), S3(5 * N), D3(5 * N);
  std::vector<double> Bn(B, B + 3 * N), SB2(3 * N), SB3(3 * N), DB3(3 * N);
  for (int s = 0; s < nst; ++s) {
    for (long long n = 0; n < N; ++n) {
      if (order == 2) bface_zone<T, 2>(B, B0.data(), BN.data(), g, n);
      if (order == 3) bface_zone<T, 3>(B, B0.data(), BN.data(), g, n);
      if (order == 4) bface_zone<T, 4>(B, B0.data(), BN.data(), g, n);
    }
    emu_recon<T>(U, W.data(), g, order, 5);
    emu_recon<T>(B0.data(), WB.data(), g, order, 3);
    for (long long n = 0; n < N; ++n) {
      if (order == 2)
        predict_zone_mhd<T, 2, 0, DEV, true, ALL, true>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, 0.0, 0.0, 0.0, 0.0, gam, emu_pc(), n);
      else if (order == 3)
        predict_zone_mhd<T, 3, 0, DEV, true, ALL, true>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, 0.0, 0.0, 0.0, 0.0, gam, emu_pc(), n);
      else
        predict_zone_mhd<T, 4, 0, DEV, true, ALL, true>(U, W.data(), B0.data(), WB.data(), BN.data(), PK.data(), g, 0.0, 0.0, 0.0, 0.0, gam, emu_pc(), n);
    }
    for (long long n = 0; n < N; ++n)
      face_flux_zone_mhd<T, RS, DEV>(U, B0.data(), PK.data(), F.data(), FE.data(), g, gam, n);
    for (long long n = 0; n < N; ++n) edge_e_zone(FE.data(), E.data(), g, n);
    const Row& r = rows[s];
    const RkStage su{r.a_n, r.a_c, r.c_l, r.a_2, r.a_3, r.c_d, Un.data(), S2.data(), S3.data(),
                     D3.data(), r.keep == 2 ? S2.data() : r.keep == 3 ? S3.data() : nullptr,
                     r.keep == 4 ? D3.data() : nullptr};
    const RkStage sb{r.a_n, r.a_c, r.c_l, r.a_2, r.a_3, r.c_d, Bn.data(), SB2.data(), SB3.data(),
                     DB3.data(), r.keep == 2 ? SB2.data() : r.keep == 3 ? SB3.data() : nullptr,
                     r.keep == 4 ? DB3.data() : nullptr};
    for (long long n = 0; n < N; ++n) rk_stage_zone(U, F.data(), su, g, dt, dx, dy, dz, n);
    for (long long n = 0; n < N; ++n) rk_stage_field_zone(B, E.data(), sb, g, dt, dx, dy, dz, n);
  }
}

extern "C" {

// Mode of the following steps (0 check, 1 limit); clears the status.
void hostemu_set_positivity(int limit) {
  g_limit = limit;
  g_bad = 0;
  g_limited = 0;
}

// Status since the last call: the check mode's violation flag and the limit
// mode's count of scaled zone polynomials; both cleared.
void hostemu_pos_status(int* bad, unsigned int* limited) {
  *bad = g_bad;
  *limited = g_limited;
  g_bad = 0;
  g_limited = 0;
}

// One SSP-RK step of ideal MHD of the host build, in place on U and B.
int hostemu_step_rk_mhd(double* U, double* B, int nx, int ny, int nz, double dx, double dy,
                        double dz, double gam, int order, int riemann, int precision, double dt) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  if (riemann == 0) {
    if (precision == 0) emu_rk_step_mhd<double, false, 0>(U, B, g, dx, dy, dz, gam, order, dt);
    else if (precision == 1) emu_rk_step_mhd<float, true, 0>(U, B, g, dx, dy, dz, gam, order, dt);
    else emu_rk_step_mhd<double, true, 0>(U, B, g, dx, dy, dz, gam, order, dt);
  } else {
    if (precision == 0) emu_rk_step_mhd<double, false, 1>(U, B, g, dx, dy, dz, gam, order, dt);
    else if (precision == 1) emu_rk_step_mhd<float, true, 1>(U, B, g, dx, dy, dz, gam, order, dt);
    else emu_rk_step_mhd<double, true, 1>(U, B, g, dx, dy, dz, gam, order, dt);
  }
  return 0;
}

// precision: 0 FP64 point form (the FP64 path), 1 FP32 deviation form (the
// mixed path), 2 FP64 deviation form (checks the deviation algebra alone).

// One MHD step of the host build, in place on U[5][N] and the face field B[3][N].
int hostemu_step_mhd(double* U, double* B, int nx, int ny, int nz, double dx, double dy,
                     double dz, double gam, int order, int form, int riemann, int precision,
                     double dt) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  if (riemann == 0) {
    if (precision == 0) emu_step_mhd<double, false, 0>(U, B, g, dx, dy, dz, gam, order, form, dt);
    else if (precision == 1) emu_step_mhd<float, true, 0>(U, B, g, dx, dy, dz, gam, order, form, dt);
    else emu_step_mhd<double, true, 0>(U, B, g, dx, dy, dz, gam, order, form, dt);
  } else {
    if (precision == 0) emu_step_mhd<double, false, 1>(U, B, g, dx, dy, dz, gam, order, form, dt);
    else if (precision == 1) emu_step_mhd<float, true, 1>(U, B, g, dx, dy, dz, gam, order, form, dt);
    else emu_step_mhd<double, true, 1>(U, B, g, dx, dy, dz, gam, order, form, dt);
  }
  return 0;
}

// |A| du of the linearized MHD solver along axis for one face (host check of
// the analytic eigen-system): ubl, ubr barycentre states, du a jump, out D.
int hostemu_mhd_dissipation(const double* ubl, const double* ubr, const double* du, int axis,
                            double gam, double* out) {
  double l[8], r[8], d[8], D[8];
  for (int v = 0; v < 8; ++v) {
    l[v] = ubl[v];
    r[v] = ubr[v];
    d[v] = du[v];
  }
  if (axis == 0) MhdEigen<double, 0>(l, r, gam).apply(d, D);
  else if (axis == 1) MhdEigen<double, 1>(l, r, gam).apply(d, D);
  else MhdEigen<double, 2>(l, r, gam).apply(d, D);
  for (int v = 0; v < 8; ++v) out[v] = D[v];
  return 0;
}

double hostemu_dt_mhd(const double* U, const double* B, int nx, int ny, int nz, double dx,
                      double dy, double dz, double gam, double cfl) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  double mx = 0.0;
  int bad = 0;
  for (long long n = 0; n < g.N; ++n) mx = fmax(mx, dt_rate_zone_mhd(U, B, g, gam, dx, dy, dz, n, bad));
  return bad ? -1.0 : cfl / mx;
}

// One step of the host build, in place on U[5][nz][ny][nx].
int hostemu_step(double* U, int nx, int ny, int nz, double dx, double dy, double dz, double gam,
                 int order, int form, int riemann, int precision, double dt) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  if (precision == 0)
    emu_step<double, false>(U, g, dx, dy, dz, gam, order, form, riemann, dt);
  else if (precision == 1)
    emu_step<float, true>(U, g, dx, dy, dz, gam, order, form, riemann, dt);
  else
    emu_step<double, true>(U, g, dx, dy, dz, gam, order, form, riemann, dt);
  return 0;
}

// One SSP-RK step of the host build (Euler), in place on U[5][nz][ny][nx].
int hostemu_step_rk(double* U, int nx, int ny, int nz, double dx, double dy, double dz,
                    double gam, int order, int riemann, int precision, double dt) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  if (precision == 0)
    emu_rk_step<double, false>(U, g, dx, dy, dz, gam, order, riemann, dt);
  else if (precision == 1)
    emu_rk_step<float, true>(U, g, dx, dy, dz, gam, order, riemann, dt);
  else
    emu_rk_step<double, true>(U, g, dx, dy, dz, gam, order, riemann, dt);
  return 0;
}

// The affine source S(u) = A u + b of the next Euler steps (A row-major 5 x
// 5, b 5 entries or NULL); A NULL removes it.
void hostemu_set_source(const double* A, const double* b) {
  g_has_src = A != nullptr;
  g_src = SourceAffine{};
  if (!A) return;
  for (int q = 0; q < 25; ++q) g_src.A[q] = A[q];
  for (int v = 0; v < 5; ++v) g_src.b[v] = b ? b[v] : 0.0;
}

// dt of the host build; returns -1 if a zone is unphysical.
double hostemu_dt(const double* U, int nx, int ny, int nz, double dx, double dy, double dz,
                  double gam, double cfl) {
  Grid g{nx, ny, nz, (long long)nx * ny * nz, (long long)nx * ny * nz, 0};
  double mx = 0.0;
  int bad = 0;
  for (long long n = 0; n < g.N; ++n) mx = fmax(mx, dt_rate_zone(U, g, gam, dx, dy, dz, n, bad));
  return bad ? -1.0 : cfl / mx;
}
}
