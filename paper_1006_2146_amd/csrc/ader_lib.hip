// Host side of libader_hip.so: the C ABI of include/ader.h, device buffers
// and the kernel sequence of one ADER-CG step.
//
// Step sequence on the context's stream (no host involvement):
//   reconstruction   k_minmod (order 2) or k_weno_sweep x, y, z (orders 3, 4);
//                    MHD first k_bface (Sec. III) and the same sweeps of b_0
//   predictor+faces  k_predict / k_predict_mhd: positivity scaling, space-time
//                    predictor, face-side packets of all six sides
//   Riemann          k_face_flux / k_face_flux_mhd: one flux per face; MHD
//                    also the edge fluxes and k_edge_e (edge fields)
//   update           k_update: eq. (6) in double; MHD k_update_mhd adds the
//                    constrained transport of eq. (8)
// and, for a CFL step, k_dt_partial + k_dt_final before it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ader.h"
#include "ader_kernels.h"

using namespace ader;

struct ader_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Grid g{};
  double lx = 1, ly = 1, lz = 1, dx = 1, dy = 1, dz = 1;
  double gamma = 1.4;
  int system = ADER_EULER;
  int order = 3, form = ADER_MODAL, riemann = ADER_HLL, precision = ADER_FP64;
  double* U = nullptr;
  bool owns_U = true;
  void* W = nullptr;
  void* PK = nullptr;
  void* F = nullptr;
  // MHD: face fields, zone field b_0, its modes, the Sec. III normal moments,
  // edge fluxes and edge fields
  double* B = nullptr;
  bool owns_B = true;
  double* B0 = nullptr;
  void* WB = nullptr;
  void* BN = nullptr;
  void* FE = nullptr;
  double* E = nullptr;
  double* d_dt = nullptr;
  double* d_partial = nullptr;
  int* d_bad = nullptr;
  int* d_status = nullptr;
  int nparts = 0;
  bool have_state = false;
  bool have_dt = false;
  size_t bytes = 0;
  // stage timing: events recorded around each stage while enabled
  bool timing = false;
  std::vector<hipEvent_t> events;
  std::vector<int> marks;  // stage of each (start, stop) event pair
};

namespace {

constexpr int kBlock = 256;
constexpr int kPredBlock = 128;

int check(hipError_t e) { return e == hipSuccess ? ADER_OK : ADER_EDEVICE; }

#define ADER_TRY(expr)            \
  do {                            \
    int _rc = (expr);             \
    if (_rc != ADER_OK) return _rc; \
  } while (0)

int launched() { return check(hipGetLastError()); }

unsigned blocks_for(long long n, int b) { return (unsigned)((n + b - 1) / b); }

int set_device(ader_ctx* c) { return check(hipSetDevice(c->device)); }

// Records an event pair around one stage when timing is on.
struct StageTimer {
  ader_ctx* c;
  int stage;
  bool on;
  StageTimer(ader_ctx* ctx, int s) : c(ctx), stage(s), on(ctx->timing) {
    if (!on) return;
    const size_t k = 2 * c->marks.size();
    while (c->events.size() < k + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      c->events.push_back(e);
    }
    (void)hipEventRecord(c->events[k], c->stream);
  }
  ~StageTimer() {
    if (!on) return;
    const size_t k = 2 * c->marks.size();
    (void)hipEventRecord(c->events[k + 1], c->stream);
    c->marks.push_back(stage);
  }
};

// zone-centred reconstruction of NVAR fields with zone averages src
template <class T, int NVAR>
int launch_sweeps(ader_ctx* c, const double* src, T* W) {
  const unsigned nb = blocks_for(c->g.N, kBlock);
  switch (c->order) {
    case 2:
      k_minmod<T, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      return launched();
    case 3:
      k_weno_sweep<T, 3, 0, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      k_weno_sweep<T, 3, 1, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      k_weno_sweep<T, 3, 2, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      return launched();
    case 4:
      k_weno_sweep<T, 4, 0, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      k_weno_sweep<T, 4, 1, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      k_weno_sweep<T, 4, 2, NVAR><<<nb, kBlock, 0, c->stream>>>(src, W, c->g);
      return launched();
  }
  return ADER_EINVAL;
}

template <class T>
int launch_recon(ader_ctx* c) {
  ADER_TRY((launch_sweeps<T, 5>(c, c->U, static_cast<T*>(c->W))));
  if (c->system != ADER_MHD) return ADER_OK;
  const unsigned nb = blocks_for(c->g.N, kBlock);
  T* BN = static_cast<T*>(c->BN);
  if (c->order == 2) k_bface<T, 2><<<nb, kBlock, 0, c->stream>>>(c->B, c->B0, BN, c->g);
  if (c->order == 3) k_bface<T, 3><<<nb, kBlock, 0, c->stream>>>(c->B, c->B0, BN, c->g);
  if (c->order == 4) k_bface<T, 4><<<nb, kBlock, 0, c->stream>>>(c->B, c->B0, BN, c->g);
  ADER_TRY(launched());
  return launch_sweeps<T, 3>(c, c->B0, static_cast<T*>(c->WB));
}

template <class T>
int launch_predict(ader_ctx* c) {
  const T* W = static_cast<const T*>(c->W);
  T* PK = static_cast<T*>(c->PK);
  const unsigned nb = blocks_for(c->g.N, kPredBlock);
  const double ix = 1.0 / c->dx, iy = 1.0 / c->dy, iz = 1.0 / c->dz;
  if (c->system == ADER_MHD) {
    const double* B0 = c->B0;
    const T* WB = static_cast<const T*>(c->WB);
    const T* BN = static_cast<const T*>(c->BN);
#define ADER_PM(O, FM) \
  k_predict_mhd<T, O, FM><<<nb, kPredBlock, 0, c->stream>>>(c->U, W, B0, WB, BN, PK, c->g, c->d_dt, ix, iy, iz, c->gamma)
    if (c->order == 2 && c->form == ADER_NODAL) ADER_PM(2, 1);
    else if (c->order == 2) ADER_PM(2, 0);
    else if (c->order == 3) ADER_PM(3, 0);
    else ADER_PM(4, 0);
#undef ADER_PM
    return launched();
  }
  if (c->order == 2 && c->form == ADER_NODAL)
    k_predict<T, 2, 1><<<nb, kPredBlock, 0, c->stream>>>(c->U, W, PK, c->g, c->d_dt, ix, iy, iz, c->gamma);
  else if (c->order == 2)
    k_predict<T, 2, 0><<<nb, kPredBlock, 0, c->stream>>>(c->U, W, PK, c->g, c->d_dt, ix, iy, iz, c->gamma);
  else if (c->order == 3)
    k_predict<T, 3, 0><<<nb, kPredBlock, 0, c->stream>>>(c->U, W, PK, c->g, c->d_dt, ix, iy, iz, c->gamma);
  else
    k_predict<T, 4, 0><<<nb, kPredBlock, 0, c->stream>>>(c->U, W, PK, c->g, c->d_dt, ix, iy, iz, c->gamma);
  return launched();
}

template <class T>
int launch_flux_update(ader_ctx* c) {
  const unsigned nb = blocks_for(c->g.N, kBlock);
  const T* PK = static_cast<const T*>(c->PK);
  double* F = static_cast<double*>(c->F);
  if (c->system == ADER_MHD) {
    double* FE = static_cast<double*>(c->FE);
    {
      StageTimer t(c, ADER_STAGE_FLUX);
      k_face_flux_mhd<T><<<nb, kBlock, 0, c->stream>>>(c->U, c->B0, PK, F, FE, c->g, c->gamma);
      ADER_TRY(launched());
      k_edge_e<<<nb, kBlock, 0, c->stream>>>(FE, c->E, c->g);
      ADER_TRY(launched());
    }
    StageTimer t(c, ADER_STAGE_UPDATE);
    k_update_mhd<<<nb, kBlock, 0, c->stream>>>(c->U, c->B, F, c->E, c->g, c->d_dt, c->dx, c->dy, c->dz);
    return launched();
  }
  {
    StageTimer t(c, ADER_STAGE_FLUX);
    if (c->riemann == ADER_HLL)
      k_face_flux<T, 0><<<nb, kBlock, 0, c->stream>>>(c->U, PK, F, c->g, c->gamma);
    else
      k_face_flux<T, 1><<<nb, kBlock, 0, c->stream>>>(c->U, PK, F, c->g, c->gamma);
    ADER_TRY(launched());
  }
  StageTimer t(c, ADER_STAGE_UPDATE);
  k_update<<<nb, kBlock, 0, c->stream>>>(c->U, F, c->g, c->d_dt, c->dx, c->dy, c->dz);
  return launched();
}

template <class T>
int launch_step(ader_ctx* c) {
  {
    StageTimer t(c, ADER_STAGE_RECON);
    ADER_TRY(launch_recon<T>(c));
  }
  {
    StageTimer t(c, ADER_STAGE_PREDICT);
    ADER_TRY(launch_predict<T>(c));
  }
  return launch_flux_update<T>(c);
}

int run_step(ader_ctx* c) {
  return c->precision == ADER_FP64 ? launch_step<double>(c) : launch_step<float>(c);
}

int queue_dt(ader_ctx* c, double cfl) {
  StageTimer t(c, ADER_STAGE_DT);
  k_dt_partial<<<c->nparts, kBlock, 0, c->stream>>>(c->U, c->system == ADER_MHD ? c->B : nullptr,
                                                    c->g, c->gamma, c->dx, c->dy, c->dz,
                                                    c->d_partial, c->d_bad);
  ADER_TRY(launched());
  k_dt_final<<<1, 1024, 0, c->stream>>>(c->d_partial, c->d_bad, c->nparts, cfl, c->d_dt,
                                        c->d_status);
  ADER_TRY(launched());
  c->have_dt = true;
  return ADER_OK;
}

int read_status(ader_ctx* c) {
  int st = 0;
  ADER_TRY(check(hipMemcpyAsync(&st, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream)));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  if (st) {
    const int zero = 0;
    ADER_TRY(check(hipMemcpyAsync(c->d_status, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream)));
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
    return ADER_ESTATE;
  }
  return ADER_OK;
}

// rho > 0, P > 0 and finite values in every zone (MHD: the zone field is
// the mean of its two face values, as in the CFL rate)
bool host_state_ok(const double* U, const double* B, const Grid& g, double gamma) {
  const long long N = g.N;
  for (long long n = 0; n < N; ++n) {
    const double r = U[n], mx = U[N + n], my = U[2 * N + n], mz = U[3 * N + n], E = U[4 * N + n];
    if (!(std::isfinite(r) && std::isfinite(mx) && std::isfinite(my) && std::isfinite(mz) &&
          std::isfinite(E)))
      return false;
    if (!(r > 0.0)) return false;
    double b2 = 0.0;
    if (B) {
      const int i = (int)(n % g.nx), j = (int)((n / g.nx) % g.ny), k = (int)(n / ((long long)g.nx * g.ny));
      const long long up[3] = {((long long)k * g.ny + j) * g.nx + (i + 1) % g.nx,
                               ((long long)k * g.ny + (j + 1) % g.ny) * g.nx + i,
                               ((long long)((k + 1) % g.nz) * g.ny + j) * g.nx + i};
      for (int d = 0; d < 3; ++d) {
        const double lo = B[d * N + n], hi = B[d * N + up[d]];
        if (!(std::isfinite(lo) && std::isfinite(hi))) return false;
        const double bm = 0.5 * (lo + hi);
        b2 += bm * bm;
      }
    }
    const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / r -
                                      b2 / (8.0 * 3.14159265358979323846));
    if (!(p > 0.0)) return false;
  }
  return true;
}

void drop_events(ader_ctx* c) {
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  c->marks.clear();
}

void free_buffers(ader_ctx* c) {
  if (c->owns_U && c->U) (void)hipFree(c->U);
  if (c->owns_B && c->B) (void)hipFree(c->B);
  if (c->B0) (void)hipFree(c->B0);
  if (c->WB) (void)hipFree(c->WB);
  if (c->BN) (void)hipFree(c->BN);
  if (c->FE) (void)hipFree(c->FE);
  if (c->E) (void)hipFree(c->E);
  if (c->W) (void)hipFree(c->W);
  if (c->PK) (void)hipFree(c->PK);
  if (c->F) (void)hipFree(c->F);
  if (c->d_dt) (void)hipFree(c->d_dt);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_bad) (void)hipFree(c->d_bad);
  if (c->d_status) (void)hipFree(c->d_status);
}

}  // namespace

extern "C" {

int ader_create(const ader_mesh* mesh, int system, int device, void* stream, ader_ctx** out) {
  if (!mesh || !out) return ADER_EINVAL;
  *out = nullptr;
  if (system != ADER_EULER && system != ADER_MHD) return ADER_EINVAL;
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return ADER_EINVAL;
  if (!(mesh->lx > 0 && mesh->ly > 0 && mesh->lz > 0)) return ADER_EINVAL;
  if (!(std::isfinite(mesh->lx) && std::isfinite(mesh->ly) && std::isfinite(mesh->lz))) return ADER_EINVAL;
  const long long N = (long long)mesh->nx * mesh->ny * mesh->nz;
  if (N > (1LL << 40)) return ADER_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ADER_EDEVICE;
  ader_ctx* c = new (std::nothrow) ader_ctx();
  if (!c) return ADER_ENOMEM;
  c->device = device;
  c->system = system;
  c->stream = static_cast<hipStream_t>(stream);
  c->g = Grid{mesh->nx, mesh->ny, mesh->nz, N};
  c->lx = mesh->lx;
  c->ly = mesh->ly;
  c->lz = mesh->lz;
  c->dx = mesh->lx / mesh->nx;
  c->dy = mesh->ly / mesh->ny;
  c->dz = mesh->lz / mesh->nz;
  c->nparts = (int)blocks_for(N, kBlock);
  if (set_device(c) != ADER_OK) {
    delete c;
    return ADER_EDEVICE;
  }
  // buffers sized for the largest case: order 4 and double work arrays
  const bool mhd = system == ADER_MHD;
  const size_t sU = sizeof(double) * 5 * (size_t)N;
  const size_t sW = sizeof(double) * 19 * 5 * (size_t)N;
  const size_t sPK = sizeof(double) * 6 * (mhd ? 32 : 15) * (size_t)N;
  const size_t sF = sizeof(double) * 3 * 5 * (size_t)N;
  const size_t s3 = sizeof(double) * 3 * (size_t)N;
  const size_t sM = mhd ? s3 * (1 + 1 + 19 + 3 + 4 + 1) : 0;  // B, B0, WB, BN, FE, E
  bool ok = hipMalloc(&c->U, sU) == hipSuccess && hipMalloc(&c->W, sW) == hipSuccess &&
            hipMalloc(&c->PK, sPK) == hipSuccess && hipMalloc(&c->F, sF) == hipSuccess &&
            (!mhd || (hipMalloc(&c->B, s3) == hipSuccess && hipMalloc(&c->B0, s3) == hipSuccess &&
                      hipMalloc(&c->WB, 19 * s3) == hipSuccess &&
                      hipMalloc(&c->BN, 3 * s3) == hipSuccess &&
                      hipMalloc(&c->FE, 4 * s3) == hipSuccess &&
                      hipMalloc(&c->E, s3) == hipSuccess)) &&
            hipMalloc(&c->d_dt, sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_partial, sizeof(double) * c->nparts) == hipSuccess &&
            hipMalloc(&c->d_bad, sizeof(int) * c->nparts) == hipSuccess &&
            hipMalloc(&c->d_status, sizeof(int)) == hipSuccess;
  if (!ok) {
    free_buffers(c);
    delete c;
    (void)hipGetLastError();
    return ADER_ENOMEM;
  }
  c->bytes = sU + sW + sPK + sF + sM + sizeof(double) * (1 + c->nparts) + sizeof(int) * (c->nparts + 1);
  const int zero = 0;
  const double no_dt = 0.0;
  if (hipMemcpy(c->d_status, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_dt, &no_dt, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    free_buffers(c);
    delete c;
    return ADER_EDEVICE;
  }
  *out = c;
  return ADER_OK;
}

int ader_set_gamma(ader_ctx* c, double gamma) {
  if (!c || !(gamma > 1.0) || !std::isfinite(gamma)) return ADER_EINVAL;
  c->gamma = gamma;
  return ADER_OK;
}

int ader_set_order(ader_ctx* c, int order, int form) {
  if (!c || order < 2 || order > 4) return ADER_EINVAL;
  if (form != ADER_MODAL && form != ADER_NODAL) return ADER_EINVAL;
  if (form == ADER_NODAL && order != 2) return ADER_EUNSUPPORTED;
  c->order = order;
  c->form = form;
  return ADER_OK;
}

int ader_set_riemann(ader_ctx* c, int riemann) {
  if (!c || (riemann != ADER_HLL && riemann != ADER_LINEARIZED)) return ADER_EINVAL;
  if (c->system == ADER_MHD && riemann != ADER_HLL) return ADER_EUNSUPPORTED;
  c->riemann = riemann;
  return ADER_OK;
}

int ader_set_precision(ader_ctx* c, int precision) {
  if (!c || (precision != ADER_FP64 && precision != ADER_MIXED)) return ADER_EINVAL;
  c->precision = precision;
  return ADER_OK;
}

int ader_set_state(ader_ctx* c, const double* U, const double* B) {
  if (!c || !U) return ADER_EINVAL;
  const bool mhd = c->system == ADER_MHD;
  if (mhd != (B != nullptr)) return ADER_EINVAL;
  if (!host_state_ok(U, B, c->g, c->gamma)) return ADER_ESTATE;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipMemcpyAsync(c->U, U, sizeof(double) * 5 * (size_t)c->g.N, hipMemcpyHostToDevice,
                                c->stream)));
  if (mhd)
    ADER_TRY(check(hipMemcpyAsync(c->B, B, sizeof(double) * 3 * (size_t)c->g.N,
                                  hipMemcpyHostToDevice, c->stream)));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  c->have_state = true;
  return ADER_OK;
}

int ader_bind_device_state(ader_ctx* c, void* dU, void* dB) {
  if (!c || !dU) return ADER_EINVAL;
  const bool mhd = c->system == ADER_MHD;
  if (mhd != (dB != nullptr)) return ADER_EINVAL;
  if (c->owns_U && c->U) (void)hipFree(c->U);
  c->U = static_cast<double*>(dU);
  c->owns_U = false;
  if (mhd) {
    if (c->owns_B && c->B) (void)hipFree(c->B);
    c->B = static_cast<double*>(dB);
    c->owns_B = false;
  }
  c->have_state = true;
  return ADER_OK;
}

int ader_get_state(ader_ctx* c, double* U, double* B) {
  if (!c || !U) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipMemcpyAsync(U, c->U, sizeof(double) * 5 * (size_t)c->g.N, hipMemcpyDeviceToHost,
                                c->stream)));
  if (B && c->system == ADER_MHD)
    ADER_TRY(check(hipMemcpyAsync(B, c->B, sizeof(double) * 3 * (size_t)c->g.N,
                                  hipMemcpyDeviceToHost, c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

int ader_compute_dt(ader_ctx* c, double cfl, double* dt_out) {
  if (!c || !(cfl > 0.0) || !std::isfinite(cfl)) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(queue_dt(c, cfl));
  if (dt_out) {
    ADER_TRY(read_status(c));
    ADER_TRY(check(hipMemcpyAsync(dt_out, c->d_dt, sizeof(double), hipMemcpyDeviceToHost, c->stream)));
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
  }
  return ADER_OK;
}

int ader_step(ader_ctx* c, double dt) {
  if (!c || !(dt > 0.0) || !std::isfinite(dt)) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  k_set_scalar<<<1, 64, 0, c->stream>>>(c->d_dt, dt);
  ADER_TRY(launched());
  c->have_dt = true;
  return run_step(c);
}

int ader_step_cfl(ader_ctx* c, double cfl) {
  if (!c || !(cfl > 0.0) || !std::isfinite(cfl)) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(queue_dt(c, cfl));
  return run_step(c);
}

int ader_get_dt(ader_ctx* c, double* dt_out) {
  if (!c || !dt_out) return ADER_EINVAL;
  if (!c->have_dt) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipMemcpyAsync(dt_out, c->d_dt, sizeof(double), hipMemcpyDeviceToHost, c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

int ader_synchronize(ader_ctx* c) {
  if (!c) return ADER_EINVAL;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  ADER_TRY(check(hipGetLastError()));
  return read_status(c);
}

int ader_set_timing(ader_ctx* c, int enable) {
  if (!c) return ADER_EINVAL;
  ADER_TRY(set_device(c));
  if (!enable) {
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
    drop_events(c);
  }
  c->marks.clear();
  c->timing = enable != 0;
  return ADER_OK;
}

int ader_stage_times(ader_ctx* c, double* ms_out, int* counts_out) {
  if (!c || !ms_out || !counts_out) return ADER_EINVAL;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  for (int s = 0; s < ADER_NSTAGES; ++s) {
    ms_out[s] = 0.0;
    counts_out[s] = 0;
  }
  for (size_t q = 0; q < c->marks.size(); ++q) {
    float ms = 0.f;
    ADER_TRY(check(hipEventElapsedTime(&ms, c->events[2 * q], c->events[2 * q + 1])));
    ms_out[c->marks[q]] += ms;
    counts_out[c->marks[q]] += 1;
  }
  c->marks.clear();
  return ADER_OK;
}

int ader_device_bytes(ader_ctx* c, double* bytes_out) {
  if (!c || !bytes_out) return ADER_EINVAL;
  *bytes_out = (double)c->bytes;
  return ADER_OK;
}

const char* ader_strerror(int code) {
  switch (code) {
    case ADER_OK: return "ok";
    case ADER_EINVAL: return "invalid argument";
    case ADER_EUNSUPPORTED: return "unsupported configuration";
    case ADER_ENOMEM: return "device allocation failed";
    case ADER_EDEVICE: return "HIP device error";
    case ADER_ESTATE: return "unphysical state (rho <= 0, P <= 0 or non-finite)";
    case ADER_ESEQ: return "call out of sequence";
  }
  return "unknown error";
}

void ader_destroy(ader_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_events(c);
  free_buffers(c);
  delete c;
}

}  // extern "C"
