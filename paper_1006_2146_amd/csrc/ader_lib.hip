// Host side of libader_hip.so: the C ABI of include/ader.h, device buffers,
// the kernel sequence of one ADER-CG step, its hipGraph and the autotuner.
//
// Step sequence on the context's stream (no host involvement), each stage
// one persistent launch over every problem of the context:
//   dt               k_dt (per-problem CFL rate, atomic max) + k_dt_final
//   reconstruction   k_minmod (order 2) or k_weno_sweep x, y, z (orders 3, 4);
//                    MHD adds k_bface (Sec. III) and the sweeps of b_0
//   predictor+faces  k_predict / k_predict_mhd: positivity scaling, space-time
//                    predictor, face-side packets of all six sides
//   Riemann          k_face_flux / k_face_flux_mhd (+ k_edge_e for MHD)
//   update           k_update: eq. (6) in double; MHD k_update_mhd adds the
//                    constrained transport of eq. (8)
// The stage launches of each (system, precision, order, form) variant live
// in their own translation unit (ader_stages.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ader_ctx.h"
#include "ader_kernels.h"

using namespace ader;

namespace {

int set_device(ader_ctx* c) { return check(hipSetDevice(c->device)); }

// The stage table of the setting (SSP-RK uses the modal tables: it has no
// predictor, so the form does not apply to it).
const StageFns* stages_of(const ader_ctx* c) {
  const int form = c->scheme == ADER_SCHEME_SSPRK ? ADER_MODAL : c->form;
#define ADER_PICK(SY, PR, OR, FM)                                                                \
  if (c->system == (#SY[0] == 'm' ? ADER_MHD : #SY[0] == 'l' ? ADER_LINADV : ADER_EULER) &&      \
      c->precision == (#PR[0] == 'm' ? ADER_MIXED : ADER_FP64) && c->order == OR && form == FM) \
    return ADER_STAGES_NAME(SY, PR, OR, FM)();
  ADER_VARIANTS(ADER_PICK)
#undef ADER_PICK
  return nullptr;
}

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

// Ghost zones of bounded problems from the current interior (before the dt
// rule and each step reads them).
int fill_ghosts(ader_ctx* c) {
  if (!c->bounded) return ADER_OK;
  // every inflow face needs its state (the faces are the same for all problems)
  for (int f = 0; f < 6; ++f)
    if (c->probs[0].bc[f] == ADER_BC_INFLOW && !((c->inflow_set >> f) & 1u)) return ADER_ESEQ;
  k_fill_ghosts<><<<grid_for(c, kClassUpdate), c->shape[kClassUpdate].block, 0, c->stream>>>(
      c->U, c->batch(), c->inflow);
  return launched();
}

int queue_dt(ader_ctx* c, double cfl) {
  StageTimer t(c, ADER_STAGE_DT);
  ADER_TRY(fill_ghosts(c));
  if (c->system == ADER_LINADV) {
    k_dt_adv<><<<(c->np() + 63) / 64, 64, 0, c->stream>>>(c->batch(), cfl, c->adv[0], c->adv[1],
                                                           c->adv[2], c->d_dt);
    ADER_TRY(launched());
    c->have_dt = true;
    return ADER_OK;
  }
  k_dt<><<<grid_for(c, kClassDt), c->shape[kClassDt].block, 0, c->stream>>>(
      c->U, c->system == ADER_MHD ? c->B : nullptr, c->batch(), c->gamma, c->d_rate, c->d_bad);
  ADER_TRY(launched());
  k_dt_final<><<<(c->np() + 63) / 64, 64, 0, c->stream>>>(c->d_rate, c->d_bad, c->np(), cfl, c->d_dt);
  ADER_TRY(launched());
  c->have_dt = true;
  return ADER_OK;
}

// The predictor layout in use: the one set, else the layout measured fastest
// without tuning: two lanes per zone for MHD at orders 3 and 4 (one kernel at
// order 3, the two-kernel form at order 4, where only it is built), one lane
// per zone and variable for Euler at order 4, one lane per zone otherwise.
bool layout_built(const ader_ctx* c, const StageFns* s, int layout) {
  if (layout == ADER_LAYOUT_ZONE2 && c->system == ADER_MHD && c->riemann == ADER_LINEARIZED)
    return false;
  switch (layout) {
    case ADER_LAYOUT_ZONE: return s->predict != nullptr;
    case ADER_LAYOUT_SPLIT: return s->predict_split != nullptr;
    case ADER_LAYOUT_SPLIT2: return s->predict_split2 != nullptr;
    case ADER_LAYOUT_ZONE2: return s->predict_zone2 != nullptr;
    case ADER_LAYOUT_ZONE_2W: return s->predict_zone_2w != nullptr;
    case ADER_LAYOUT_PAIR: return s->predict_pair != nullptr;
    case ADER_LAYOUT_PAIR2: return s->predict_pair2 != nullptr;
    case ADER_LAYOUT_PAIR_SPLIT: return s->predict_pair_split != nullptr;
    case ADER_LAYOUT_FUSED: return s->predict_fused != nullptr;
  }
  return false;
}

int layout_of(const ader_ctx* c, const StageFns* s) {
  // the source instances: one lane per zone at orders 2 and 3, lane-split at 4
  if (c->has_source) return c->order == 4 ? ADER_LAYOUT_SPLIT : ADER_LAYOUT_ZONE;
  if (c->layout >= 0 && layout_built(c, s, c->layout)) return c->layout;
  if (s->predict_pair && c->system == ADER_MHD) return ADER_LAYOUT_PAIR;
  if (s->predict_pair_split && c->system == ADER_MHD) return ADER_LAYOUT_PAIR_SPLIT;
  if (s->predict_split && c->order == 4) return ADER_LAYOUT_SPLIT;
  return ADER_LAYOUT_ZONE;
}

int queue_predict(ader_ctx* c, const StageFns* s) {
  if (c->has_source) return s->predict_src ? s->predict_src(c) : ADER_EUNSUPPORTED;
  switch (layout_of(c, s)) {
    case ADER_LAYOUT_SPLIT: return s->predict_split(c);
    case ADER_LAYOUT_SPLIT2: return s->predict_split2(c);
    case ADER_LAYOUT_ZONE2: return s->predict_zone2(c);
    case ADER_LAYOUT_ZONE_2W: return s->predict_zone_2w(c);
    case ADER_LAYOUT_PAIR: return s->predict_pair(c);
    case ADER_LAYOUT_PAIR2: return s->predict_pair2(c);
    case ADER_LAYOUT_PAIR_SPLIT: return s->predict_pair_split(c);
    case ADER_LAYOUT_FUSED: return s->predict_fused(c);
    default: return s->predict ? s->predict(c) : ADER_EUNSUPPORTED;
  }
}

// face fluxes and update in one launch (ctx flux_fused())
int queue_flux_update(ader_ctx* c) {
  const long long cap = (long long)c->shape[kClassFlux].blocks_per_cu * c->num_cus;
  const unsigned g = (unsigned)(c->nfutiles < cap ? c->nfutiles : cap);
  const dim3 grid(g < 1 ? 1 : g), block(kFuTX * kFuTY);
  const bool hll = c->riemann == ADER_HLL;
  if (c->precision == ADER_MIXED) {
    const float* PK = static_cast<const float*>(c->PK);
    if (hll)
      k_flux_update<float, 0><<<grid, block, 0, c->stream>>>(c->U, c->keep_avg(), PK, c->batch(),
                                                             c->d_fu_base, c->d_dt, c->gamma);
    else
      k_flux_update<float, 1><<<grid, block, 0, c->stream>>>(c->U, c->keep_avg(), PK, c->batch(),
                                                             c->d_fu_base, c->d_dt, c->gamma);
  } else {
    const double* PK = static_cast<const double*>(c->PK);
    if (hll)
      k_flux_update<double, 0><<<grid, block, 0, c->stream>>>(c->U, nullptr, PK, c->batch(),
                                                              c->d_fu_base, c->d_dt, c->gamma);
    else
      k_flux_update<double, 1><<<grid, block, 0, c->stream>>>(c->U, nullptr, PK, c->batch(),
                                                               c->d_fu_base, c->d_dt, c->gamma);
  }
  return launched();
}

int queue_flux(ader_ctx* c, const StageFns* s) {
  return c->flux_fused() ? queue_flux_update(c) : s->flux(c);
}

// a no-op when the fused kernel has updated already
int queue_update(ader_ctx* c, const StageFns* s) {
  if (c->flux_fused()) return ADER_OK;
  if (c->has_source) return s->update_src ? s->update_src(c) : ADER_EUNSUPPORTED;
  return s->update(c);
}

// SSP-RK weights of eq. (18), (19) and (20), one row per stage: U <- a_n Un
// + a_c U + c_l dt L(U) + a_2 U^(2) + a_3 U^(3) + c_d dt L(U^(3)); the flags
// keep U^(2), U^(3) and dt L(U^(3)) for the last stage of (20).
struct RkRow {
  double a_n, a_c, c_l, a_2, a_3, c_d;
  int keep;   // 2: keep the result as U^(2); 3: as U^(3); 4: keep dt L
};
constexpr RkRow kRk2[] = {{0, 1, 1, 0, 0, 0, 0}, {0.5, 0.5, 0.5, 0, 0, 0, 0}};
constexpr RkRow kRk3[] = {{0, 1, 1, 0, 0, 0, 0}, {0.75, 0.25, 0.25, 0, 0, 0, 0},
                          {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 0, 0, 0, 0}};
constexpr RkRow kRk54[] = {
    {0, 1, 0.39175222700392, 0, 0, 0, 0},
    {0.44437049406734, 0.55562950593266, 0.36841059262959, 0, 0, 0, 2},
    {0.62010185138540, 0.37989814861460, 0.25189177424738, 0, 0, 0, 3},
    {0.17807995410773, 0.82192004589227, 0.54497475021237, 0, 0, 0, 4},
    {0.00683325884039, 0.34833675773694, 0.22600748319395, 0.51723167208978, 0.12759831133288,
     0.08460416338212, 0}};

// One SSP-RK step (Sec. II.d): the starting state saved, then per stage the
// reconstruction, the side packets of the spatial polynomial, the face
// fluxes and the stage combination, all on the stream.
int queue_rk_step(ader_ctx* c, const StageFns* s) {
  if (!s->rk_sides) return ADER_EUNSUPPORTED;
  const RkRow* rows = c->order == 2 ? kRk2 : c->order == 3 ? kRk3 : kRk54;
  const int nst = c->order == 2 ? 2 : c->order == 3 ? 3 : 5;
  const long long row = 5 * c->S, brow = 3 * c->S;
  const bool mhd = c->system == ADER_MHD;
  double* Un = c->RK;
  double* S2 = c->RK + row;
  double* S3 = c->RK + 2 * row;
  double* D3 = c->RK + 3 * row;
  // MHD: the same four arrays for the face fields after the hydro ones
  double* Bn = c->RK + 4 * row;
  double* SB2 = Bn + brow;
  double* SB3 = Bn + 2 * brow;
  double* DB3 = Bn + 3 * brow;
  const unsigned gu = grid_for(c, kClassUpdate);
  const int bu = c->shape[kClassUpdate].block;
  {
    StageTimer t(c, ADER_STAGE_UPDATE);
    k_copy_state<><<<gu, bu, 0, c->stream>>>(c->U, Un, 5, c->batch());
    ADER_TRY(launched());
    if (mhd) {
      k_copy_state<><<<gu, bu, 0, c->stream>>>(c->B, Bn, 3, c->batch());
      ADER_TRY(launched());
    }
  }
  for (int k = 0; k < nst; ++k) {
    const RkRow& r = rows[k];
    {
      StageTimer t(c, ADER_STAGE_RECON);
      ADER_TRY(s->recon(c));
    }
    {
      StageTimer t(c, ADER_STAGE_PREDICT);
      ADER_TRY(s->rk_sides(c));
    }
    {
      StageTimer t(c, ADER_STAGE_FLUX);
      ADER_TRY(s->flux(c));
    }
    StageTimer t(c, ADER_STAGE_UPDATE);
    const RkStage st{r.a_n, r.a_c, r.c_l, r.a_2, r.a_3, r.c_d, Un, S2, S3, D3,
                     r.keep == 2 ? S2 : r.keep == 3 ? S3 : nullptr, r.keep == 4 ? D3 : nullptr};
    k_rk_stage<><<<gu, bu, 0, c->stream>>>(c->U, c->F, st, c->batch(), c->d_dt);
    ADER_TRY(launched());
    if (mhd) {
      const RkStage sb{r.a_n, r.a_c, r.c_l, r.a_2, r.a_3, r.c_d, Bn, SB2, SB3, DB3,
                       r.keep == 2 ? SB2 : r.keep == 3 ? SB3 : nullptr,
                       r.keep == 4 ? DB3 : nullptr};
      k_rk_stage_field<><<<gu, bu, 0, c->stream>>>(c->B, c->E, sb, c->batch(), c->d_dt);
      ADER_TRY(launched());
    }
  }
  return ADER_OK;
}

int queue_step(ader_ctx* c) {
  const StageFns* s = stages_of(c);
  if (!s) return ADER_EUNSUPPORTED;
  if (c->scheme == ADER_SCHEME_SSPRK)
    return (c->has_source || c->bounded) ? ADER_EUNSUPPORTED : queue_rk_step(c, s);
  // the fused layout reconstructs inside its predictor kernel
  if (layout_of(c, s) != ADER_LAYOUT_FUSED) {
    StageTimer t(c, ADER_STAGE_RECON);
    ADER_TRY(s->recon(c));
  }
  {
    StageTimer t(c, ADER_STAGE_PREDICT);
    ADER_TRY(queue_predict(c, s));
  }
  {
    StageTimer t(c, ADER_STAGE_FLUX);
    ADER_TRY(queue_flux(c, s));
  }
  StageTimer t(c, ADER_STAGE_UPDATE);
  return queue_update(c, s);
}

void drop_graph(ader_ctx* c);

// Work arrays for the current order and precision: W (modes 2..L_S of the 5
// hydro variables), PK (six side packets), and for MHD WB (modes of the zone
// field) and BN (its Sec. III normal moments), in the bulk type (double or
// float).  Grown (freed and allocated again) when a setting needs more; never
// called while a stream capture is open.
int ensure_work(ader_ctx* c) {
  const size_t Z = (size_t)c->S;
  const size_t t = c->precision == ADER_FP64 ? sizeof(double) : sizeof(float);
  const size_t ls = c->order == 2 ? 4 : c->order == 3 ? 10 : 20;
  const bool mhd = c->system == ADER_MHD;
  const size_t ne = c->order == 2 ? 1 : c->order == 3 ? 5 : 15;   // evolutionary modes
  // the two-kernel pair layout's mode and factor buffers, for the layout
  // the step will run (set explicitly or the default of the setting)
  const StageFns* st = stages_of(c);
  const bool split = mhd && c->order >= 3 && st && layout_of(c, st) == ADER_LAYOUT_PAIR_SPLIT;
  const size_t need[8] = {t * (ls - 1) * 5 * Z, t * 6 * (mhd ? kMhdSlots : 15) * Z,
                          mhd ? t * (ls - 1) * 3 * Z : 0, mhd ? t * 3 * 3 * Z : 0,
                          c->scheme == ADER_SCHEME_SSPRK ? sizeof(double) * 4 * (mhd ? 8 : 5) * Z
                                                         : 0,
                          split ? t * ne * 8 * Z : 0, split ? sizeof(double) * 2 * Z : 0,
                          c->has_source ? sizeof(double) * 5 * Z : 0};
  void** buf[8] = {&c->W,  &c->PK, &c->WB,           &c->BN, (void**)&c->RK,
                   &c->EM, (void**)&c->TH, (void**)&c->SB};
  for (int q = 0; q < 8; ++q) {
    if (need[q] <= c->work_bytes[q]) continue;
    if (*buf[q]) {
      // a captured step holds the old address: rebuild it on its next use
      ADER_TRY(check(hipStreamSynchronize(c->stream)));
      drop_graph(c);
      (void)hipFree(*buf[q]);
      *buf[q] = nullptr;
      c->work_bytes[q] = 0;
    }
    if (hipMalloc(buf[q], need[q]) != hipSuccess) {
      *buf[q] = nullptr;
      (void)hipGetLastError();
      c->bytes = c->fixed_bytes;
      for (size_t w : c->work_bytes) c->bytes += w;
      return ADER_ENOMEM;
    }
    c->work_bytes[q] = need[q];
  }
  c->bytes = c->fixed_bytes;
  for (size_t w : c->work_bytes) c->bytes += w;
  return ADER_OK;
}

// Everything a captured step depends on besides the device buffers' contents.
unsigned long long config_key(const ader_ctx* c) {
  unsigned long long k = (unsigned long long)c->order;
  k = k * 3 + (unsigned long long)c->form;
  k = k * 3 + (unsigned long long)c->riemann;
  k = k * 3 + (unsigned long long)c->precision;
  k = k * 3 + (unsigned long long)(c->layout + 1);
  k = k * 3 + (unsigned long long)(c->recon_mode + 1);
  k = k * 3 + (unsigned long long)(c->flux_mode + 1);
  k = k * 3 + (unsigned long long)c->scheme;
  k = k * 3 + (unsigned long long)c->positivity;
  k = k * 1000003 + c->source_version;
  k = k * 1000003 + c->inflow_version;
  for (int q = 0; q < kNumClasses; ++q) k = k * 1031 + (unsigned long long)c->shape[q].block * 37 +
                                            (unsigned long long)c->shape[q].blocks_per_cu;
  k ^= (unsigned long long)(uintptr_t)c->U * 0x9e3779b97f4a7c15ull;
  k ^= (unsigned long long)(uintptr_t)c->B * 0xc2b2ae3d27d4eb4full;
  k ^= (unsigned long long)(uintptr_t)c->W * 0xd6e8feb86659fd93ull;
  k ^= (unsigned long long)(uintptr_t)c->PK * 0xa0761d6478bd642full;
  k ^= (unsigned long long)(uintptr_t)c->SB * 0xe7037ed1a0b428dbull;
  for (int d = 0; d < 3; ++d) {
    unsigned long long a;
    std::memcpy(&a, &c->adv[d], sizeof a);
    k = k * 1099511628211ull ^ a;
  }
  unsigned long long g;
  std::memcpy(&g, &c->gamma, sizeof g);
  return k ^ (g * 0x165667b19e3779f9ull);
}

void drop_graph(ader_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  c->graph_exec = nullptr;
}

// One CFL step: replayed from a hipGraph when graph mode is on (captured on
// first use and whenever the configuration, cfl or bound buffers change),
// launched eagerly otherwise or while stage timing is on.
int run_step_cfl(ader_ctx* c, double cfl) {
  ADER_TRY(ensure_work(c));
  if (!c->use_graph || c->timing) {
    ADER_TRY(queue_dt(c, cfl));
    return queue_step(c);
  }
  const unsigned long long key = config_key(c);
  if (!c->graph_exec || c->graph_cfl != cfl || c->graph_key != key) {
    drop_graph(c);
    ADER_TRY(check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)));
    int rc = queue_dt(c, cfl);
    if (rc == ADER_OK) rc = queue_step(c);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (rc != ADER_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    ADER_TRY(check(e));
    const hipError_t ei = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    ADER_TRY(check(ei));
    c->graph_cfl = cfl;
    c->graph_key = key;
  }
  c->have_dt = true;
  return check(hipGraphLaunch(c->graph_exec, c->stream));
}

// Copies the per-problem flags back; any set flag is ADER_ESTATE (and the
// flags are cleared).
int read_status(ader_ctx* c) {
  std::vector<int> bad(c->np(), 0);
  ADER_TRY(check(hipMemcpyAsync(bad.data(), c->d_bad, sizeof(int) * bad.size(),
                                hipMemcpyDeviceToHost, c->stream)));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  if (std::any_of(bad.begin(), bad.end(), [](int b) { return b != 0; })) {
    ADER_TRY(check(hipMemsetAsync(c->d_bad, 0, sizeof(int) * bad.size(), c->stream)));
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
    return ADER_ESTATE;
  }
  return ADER_OK;
}

// rho > 0, P > 0 and finite values in every zone of one problem stored with
// stride S at base (MHD: the zone field is the mean of its two face values,
// as in the CFL rate); for linear advection (physical false) finite values
bool host_state_ok(const double* U, const double* B, const Problem& pr, long long S,
                   double gamma, bool physical = true) {
  for (long long l = 0; l < pr.N; ++l) {
    const long long n = pr.base + l;
    const double r = U[n], mx = U[S + n], my = U[2 * S + n], mz = U[3 * S + n], E = U[4 * S + n];
    if (!(std::isfinite(r) && std::isfinite(mx) && std::isfinite(my) && std::isfinite(mz) &&
          std::isfinite(E)))
      return false;
    if (!physical) continue;
    if (!(r > 0.0)) return false;
    double b2 = 0.0;
    if (B) {
      const int i = (int)(l % pr.nx), j = (int)((l / pr.nx) % pr.ny),
                k = (int)(l / ((long long)pr.nx * pr.ny));
      const long long up[3] = {pr.base + ((long long)k * pr.ny + j) * pr.nx + (i + 1) % pr.nx,
                               pr.base + ((long long)k * pr.ny + (j + 1) % pr.ny) * pr.nx + i,
                               pr.base + ((long long)((k + 1) % pr.nz) * pr.ny + j) * pr.nx + i};
      for (int d = 0; d < 3; ++d) {
        const double lo = B[d * S + n], hi = B[d * S + up[d]];
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
  for (void* p : {(void*)c->B0, c->WB, c->BN, (void*)c->FE, (void*)c->E, c->W, c->PK, (void*)c->F,
                  (void*)c->RK, c->EM, (void*)c->TH, (void*)c->SB,
                  (void*)c->d_dt, (void*)c->d_rate, (void*)c->d_bad, (void*)c->d_limited,
                  (void*)c->d_probs,
                  (void*)c->d_tile_base, (void*)c->d_ftile_base, (void*)c->d_xytile_base, (void*)c->d_fu_base, (void*)c->d_seg_base, (void*)c->d_diag_base,
                  (void*)c->d_diag})
    if (p) (void)hipFree(p);
}

bool mesh_ok(const ader_mesh& m) {
  return m.nx >= 1 && m.ny >= 1 && m.nz >= 1 && m.lx > 0 && m.ly > 0 && m.lz > 0 &&
         std::isfinite(m.lx) && std::isfinite(m.ly) && std::isfinite(m.lz) &&
         (long long)m.nx * m.ny * m.nz <= (1LL << 40);
}

// Context for n independent problems stored one after the other.
int create(int n, const ader_mesh* meshes, int system, int device, void* stream, ader_ctx** out) {
  if (!meshes || !out || n < 1 || n > (1 << 20)) return ADER_EINVAL;
  *out = nullptr;
  if (system != ADER_EULER && system != ADER_MHD && system != ADER_LINADV) return ADER_EINVAL;
  long long S = 0;
  for (int q = 0; q < n; ++q) {
    if (!mesh_ok(meshes[q])) return ADER_EINVAL;
    S += (long long)meshes[q].nx * meshes[q].ny * meshes[q].nz;
  }
  if (S > (1LL << 40)) return ADER_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ADER_EDEVICE;
  ader_ctx* c = new (std::nothrow) ader_ctx();
  if (!c) return ADER_ENOMEM;
  c->device = device;
  c->system = system;
  c->stream = static_cast<hipStream_t>(stream);
  c->S = S;
  c->S_user = S;
  long long base = 0;
  for (int q = 0; q < n; ++q) {
    const ader_mesh& m = meshes[q];
    Problem pr{};
    pr.nx = m.nx;
    pr.ny = m.ny;
    pr.nz = m.nz;
    pr.N = (long long)m.nx * m.ny * m.nz;
    pr.base = base;
    pr.dx = m.lx / m.nx;
    pr.dy = m.ly / m.ny;
    pr.dz = m.lz / m.nz;
    pr.ux = m.nx;
    pr.uy = m.ny;
    pr.uz = m.nz;
    base += pr.N;
    c->probs.push_back(pr);
  }
  c->set_flags.assign(n, 0);
  if (set_device(c) != ADER_OK) {
    delete c;
    return ADER_EDEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    c->num_cus = cus;
  // state, fluxes and per-problem scalars now; the work arrays (modes,
  // packets) are sized for the order and precision in use at the first step
  const bool mhd = system == ADER_MHD;
  const size_t Z = (size_t)S;
  const size_t sU = sizeof(double) * 5 * Z;
  const size_t sF = sizeof(double) * 3 * 5 * Z;
  const size_t s3 = sizeof(double) * 3 * Z;
  const size_t sM = mhd ? s3 * (1 + 1 + 4 + 1) : 0;  // B, B0, FE, E
  const size_t sP = sizeof(Problem) * n, sD = sizeof(double) * n;
  bool ok = hipMalloc(&c->U, sU) == hipSuccess && hipMalloc(&c->F, sF) == hipSuccess &&
            (!mhd || (hipMalloc(&c->B, s3) == hipSuccess && hipMalloc(&c->B0, s3) == hipSuccess &&
                      hipMalloc(&c->FE, 4 * s3) == hipSuccess &&
                      hipMalloc(&c->E, s3) == hipSuccess)) &&
            hipMalloc(&c->d_probs, sP) == hipSuccess && hipMalloc(&c->d_dt, sD) == hipSuccess &&
            hipMalloc(&c->d_rate, sizeof(unsigned long long) * n) == hipSuccess &&
            hipMalloc(&c->d_bad, sizeof(int) * 2 * n) == hipSuccess &&
            hipMalloc(&c->d_limited, sizeof(unsigned int) * 2 * n) == hipSuccess &&
            hipMalloc(&c->d_tile_base, sizeof(long long) * (n + 1)) == hipSuccess &&
            hipMalloc(&c->d_ftile_base, sizeof(long long) * (n + 1)) == hipSuccess &&
            hipMalloc(&c->d_xytile_base, sizeof(long long) * (n + 1)) == hipSuccess &&
            hipMalloc(&c->d_fu_base, sizeof(long long) * (n + 1)) == hipSuccess &&
            hipMalloc(&c->d_seg_base, sizeof(long long) * (n + 1)) == hipSuccess &&
            hipMalloc(&c->d_diag_base, sizeof(long long) * (n + 1)) == hipSuccess;
  if (!ok) {
    free_buffers(c);
    delete c;
    (void)hipGetLastError();
    return ADER_ENOMEM;
  }
  c->fixed_bytes = sU + sF + sM + sP + 2 * sD + (sizeof(int) + sizeof(unsigned int)) * 2 * n +
                   6 * sizeof(long long) * (n + 1);
  c->bytes = c->fixed_bytes;
  // reconstruction tiles of kTile^3 zones per problem
  std::vector<long long> tile_base(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    const Problem& pr = c->probs[q];
    tile_base[q + 1] = tile_base[q] + (long long)((pr.nx + kTile - 1) / kTile) *
                                          ((pr.ny + kTile - 1) / kTile) * ((pr.nz + kTile - 1) / kTile);
  }
  c->ntiles = tile_base[n];
  // tiles of the fused reconstruction+predictor: kTile x kTile x kFusedTZ
  std::vector<long long> ftile_base(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    const Problem& pr = c->probs[q];
    ftile_base[q + 1] = ftile_base[q] + (long long)((pr.nx + kTile - 1) / kTile) *
                                            ((pr.ny + kTile - 1) / kTile) *
                                            ((pr.nz + kFusedTZ - 1) / kFusedTZ);
  }
  c->nftiles = ftile_base[n];
  // segments of kMarchSeg planes of the x-y columns of kMarchTile x kMarchTile
  // zones of the z-marching reconstruction
  std::vector<long long> xytile_base(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    const Problem& pr = c->probs[q];
    xytile_base[q + 1] = xytile_base[q] + (long long)((pr.nx + kMarchTile - 1) / kMarchTile) *
                                              ((pr.ny + kMarchTile - 1) / kMarchTile) *
                                              ((pr.nz + kMarchSeg - 1) / kMarchSeg);
  }
  c->nxytiles = xytile_base[n];
  // work items of the fused face-flux+update kernel: kFuTX x kFuTY columns
  // of kFuSeg planes
  std::vector<long long> fu_base(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    const Problem& pr = c->probs[q];
    fu_base[q + 1] = fu_base[q] + (long long)((pr.nx + kFuTX - 1) / kFuTX) *
                                      ((pr.ny + kFuTY - 1) / kFuTY) * ((pr.nz + kFuSeg - 1) / kFuSeg);
  }
  c->nfutiles = fu_base[n];
  // z-column segments of kZSeg planes per (i, j) column
  std::vector<long long> seg_base(n + 1, 0);
  for (int q = 0; q < n; ++q) {
    const Problem& pr = c->probs[q];
    seg_base[q + 1] = seg_base[q] + (long long)pr.nx * pr.ny * ((pr.nz + kZSeg - 1) / kZSeg);
  }
  c->nsegs = seg_base[n];
  // diagnostics tiles of kDiagTile zones per problem
  std::vector<long long> diag_base(n + 1, 0);
  for (int q = 0; q < n; ++q)
    diag_base[q + 1] = diag_base[q] + (c->probs[q].N + kDiagTile - 1) / kDiagTile;
  c->ndiag_tiles = diag_base[n];
  if (hipMemcpy(c->d_tile_base, tile_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_ftile_base, ftile_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_xytile_base, xytile_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_fu_base, fu_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_diag_base, diag_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_seg_base, seg_base.data(), sizeof(long long) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_probs, c->probs.data(), sP, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->d_dt, 0, sD) != hipSuccess ||
      hipMemset(c->d_rate, 0, sizeof(unsigned long long) * n) != hipSuccess ||
      hipMemset(c->d_bad, 0, sizeof(int) * 2 * n) != hipSuccess ||
      hipMemset(c->d_limited, 0, sizeof(unsigned int) * 2 * n) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    free_buffers(c);
    delete c;
    return ADER_EDEVICE;
  }
  *out = c;
  return ADER_OK;
}

// Copy problem q's host arrays (U[5][N], B[3][N]) into the batch layout.
// The caller's view of a bounded problem: its interior, at base ub of rows
// of the caller's stride.
Problem user_view(const Problem& pr, long long ub) {
  Problem u = pr;
  u.nx = pr.ux;
  u.ny = pr.uy;
  u.nz = pr.uz;
  u.N = (long long)pr.ux * pr.uy * pr.uz;
  u.base = ub;
  return u;
}

// interior rows between the caller's layout (rows of stride us, problem at
// ub) and a padded host copy [5][N] of the problem
void pack_interior(const Problem& pr, const double* src, long long us, long long ub, double* dst) {
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < pr.uz; ++k)
      for (int j = 0; j < pr.uy; ++j)
        std::memcpy(dst + v * pr.N + ((long long)(k + pr.gz) * pr.ny + j + pr.gy) * pr.nx + pr.gx,
                    src + v * us + ub + ((long long)k * pr.uy + j) * pr.ux,
                    sizeof(double) * pr.ux);
}

void unpack_interior(const Problem& pr, const double* src, double* dst, long long us, long long ub) {
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < pr.uz; ++k)
      for (int j = 0; j < pr.uy; ++j)
        std::memcpy(dst + v * us + ub + ((long long)k * pr.uy + j) * pr.ux,
                    src + v * pr.N + ((long long)(k + pr.gz) * pr.ny + j + pr.gy) * pr.nx + pr.gx,
                    sizeof(double) * pr.ux);
}

int put_problem(ader_ctx* c, int q, const double* U, const double* B) {
  const Problem& pr = c->probs[q];
  const size_t bytes = sizeof(double) * (size_t)pr.N;
  for (int v = 0; v < 5; ++v)
    ADER_TRY(check(hipMemcpyAsync(c->U + v * c->S + pr.base, U + v * pr.N, bytes,
                                  hipMemcpyHostToDevice, c->stream)));
  if (B)
    for (int d = 0; d < 3; ++d)
      ADER_TRY(check(hipMemcpyAsync(c->B + d * c->S + pr.base, B + d * pr.N, bytes,
                                    hipMemcpyHostToDevice, c->stream)));
  return ADER_OK;
}

int get_problem(ader_ctx* c, int q, double* U, double* B) {
  const Problem& pr = c->probs[q];
  const size_t bytes = sizeof(double) * (size_t)pr.N;
  for (int v = 0; v < 5; ++v)
    ADER_TRY(check(hipMemcpyAsync(U + v * pr.N, c->U + v * c->S + pr.base, bytes,
                                  hipMemcpyDeviceToHost, c->stream)));
  if (B && c->system == ADER_MHD)
    for (int d = 0; d < 3; ++d)
      ADER_TRY(check(hipMemcpyAsync(B + d * pr.N, c->B + d * c->S + pr.base, bytes,
                                    hipMemcpyDeviceToHost, c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

// ---------------------------------------------------------------------------
// Autotuner: for each kernel class, time each candidate launch shape on the
// context's own problems and configuration (HIP events around a few launches
// of that stage alone) and keep the fastest.  The state is saved first and
// restored at the end, so tuning does not advance the solution.
// ---------------------------------------------------------------------------
constexpr int kNumLayouts = 9;
constexpr LaunchShape kCandidates[] = {{64, 4}, {64, 8}, {64, 16}, {128, 2}, {128, 4}, {128, 8},
                                       {256, 1}, {256, 2}, {256, 4}, {256, 8}, {256, 16}};

int time_stage(ader_ctx* c, int cls, const StageFns* s, int reps, float* ms) {
  hipEvent_t e0, e1;
  ADER_TRY(check(hipEventCreate(&e0)));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ADER_EDEVICE;
  }
  int rc = check(hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps && rc == ADER_OK; ++r) {
    switch (cls) {
      case kClassDt: rc = queue_dt(c, 0.3); break;
      case kClassRecon: rc = s->recon(c); break;
      case kClassPredict: rc = queue_predict(c, s); break;
      case kClassFlux: rc = queue_flux(c, s); break;
      default: rc = queue_update(c, s); break;
    }
  }
  if (rc == ADER_OK) rc = check(hipEventRecord(e1, c->stream));
  if (rc == ADER_OK) rc = check(hipEventSynchronize(e1));
  if (rc == ADER_OK) rc = check(hipEventElapsedTime(ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// the update's time at its fastest launch shape (the shape is kept)
int best_update_ms(ader_ctx* c, const StageFns* s, int reps, float* out) {
  const LaunchShape keep = c->shape[kClassUpdate];
  float best = 1e30f;
  int rc = ADER_OK;
  for (const LaunchShape& cand : kCandidates) {
    c->shape[kClassUpdate] = cand;
    float ms = 0.f;
    rc = time_stage(c, kClassUpdate, s, 1, &ms);
    if (rc == ADER_OK) rc = time_stage(c, kClassUpdate, s, reps, &ms);
    if (rc != ADER_OK) break;
    best = ms < best ? ms : best;
  }
  c->shape[kClassUpdate] = keep;
  *out = best;
  return rc;
}

int autotune(ader_ctx* c, int reps) {
  const StageFns* s = stages_of(c);
  if (!s) return ADER_EUNSUPPORTED;
  ADER_TRY(ensure_work(c));
  const bool mhd = c->system == ADER_MHD;
  const size_t bU = sizeof(double) * 5 * (size_t)c->S, bB = sizeof(double) * 3 * (size_t)c->S;
  double *sU = nullptr, *sB = nullptr, *sdt = nullptr;
  const size_t bD = sizeof(double) * c->np();
  if (hipMalloc(&sU, bU) != hipSuccess || hipMalloc(&sdt, bD) != hipSuccess ||
      (mhd && hipMalloc(&sB, bB) != hipSuccess)) {
    if (sU) (void)hipFree(sU);
    if (sdt) (void)hipFree(sdt);
    (void)hipGetLastError();
    return ADER_ENOMEM;
  }
  int rc = check(hipMemcpyAsync(sU, c->U, bU, hipMemcpyDeviceToDevice, c->stream));
  if (rc == ADER_OK && mhd) rc = check(hipMemcpyAsync(sB, c->B, bB, hipMemcpyDeviceToDevice, c->stream));
  if (rc == ADER_OK) rc = check(hipMemcpyAsync(sdt, c->d_dt, bD, hipMemcpyDeviceToDevice, c->stream));
  const bool timing = c->timing;
  c->timing = false;
  // one full step fills every work buffer the single stages read
  if (rc == ADER_OK) rc = queue_dt(c, 0.3);
  if (rc == ADER_OK) rc = queue_step(c);
  // the update changes the state in place: tune it (and dt) last
  const int order_of_classes[kNumClasses] = {kClassRecon, kClassPredict, kClassFlux, kClassDt,
                                             kClassUpdate};
  // the fused layout's predictor includes the reconstruction: the other
  // layouts are compared with the tuned reconstruction's time added; the
  // fused face-flux+update kernel is compared with the two kernels' sum
  float recon_ms = 0.f, update_ms = 0.f;
  const bool fusable =
      c->system == ADER_EULER && !c->has_source && c->scheme == ADER_SCHEME_ADER;
  for (int qi = 0; qi < kNumClasses && rc == ADER_OK; ++qi) {
    const int cls = order_of_classes[qi];
    LaunchShape best = c->shape[cls];
    int best_layout = c->layout;
    float best_ms = 1e30f;
    // the predictor also tries its layouts, the reconstruction its modes
    int best_recon = c->recon_mode;
    int best_flux = c->flux_mode;
    const int nlayouts = cls == kClassPredict ? kNumLayouts
                         : cls == kClassRecon ? 4
                         : (cls == kClassFlux && fusable) ? 2
                                                           : 1;
    for (int lay = 0; lay < nlayouts && rc == ADER_OK; ++lay) {
      if (cls == kClassPredict) {
        if (!layout_built(c, s, lay)) continue;
        c->layout = lay;
        rc = ensure_work(c);   // a layout may need buffers of its own
        if (rc != ADER_OK) break;
      }
      if (cls == kClassRecon) {
        if (lay != ADER_RECON_SWEEPS && c->order < 3) continue;
        c->recon_mode = lay;
      }
      if (cls == kClassFlux && nlayouts == 2) {
        c->flux_mode = lay;
        // separate: the update's best time joins; fused: one predictor launch
        // first keeps the zone averages the fused kernel reads
        rc = lay == ADER_FLUX_SEPARATE ? best_update_ms(c, s, reps, &update_ms)
                                       : queue_predict(c, s);
        if (rc != ADER_OK) break;
      }
      for (const LaunchShape& cand : kCandidates) {
        c->shape[cls] = cand;
        float ms = 0.f;
        rc = time_stage(c, cls, s, 1, &ms);  // warm-up
        if (rc == ADER_OK) rc = time_stage(c, cls, s, reps, &ms);
        if (rc != ADER_OK) break;
        if (cls == kClassPredict && c->layout != ADER_LAYOUT_FUSED) ms += recon_ms;
        if (cls == kClassFlux && nlayouts == 2 && lay == ADER_FLUX_SEPARATE) ms += update_ms;
        if (ms < best_ms) {
          best_ms = ms;
          best = cand;
          best_layout = c->layout;
          best_recon = c->recon_mode;
          best_flux = c->flux_mode;
        }
      }
    }
    c->shape[cls] = best;
    c->layout = best_layout;
    c->recon_mode = best_recon;
    c->flux_mode = best_flux;
    if (cls == kClassRecon) recon_ms = best_ms;
  }
  c->timing = timing;
  // restore the state, dt and clear the flags the trial steps may have set
  const int rc2 = check(hipMemcpyAsync(c->U, sU, bU, hipMemcpyDeviceToDevice, c->stream));
  if (mhd) (void)hipMemcpyAsync(c->B, sB, bB, hipMemcpyDeviceToDevice, c->stream);
  (void)hipMemcpyAsync(c->d_dt, sdt, bD, hipMemcpyDeviceToDevice, c->stream);
  (void)hipMemsetAsync(c->d_bad, 0, sizeof(int) * c->np(), c->stream);
  (void)hipMemsetAsync(c->d_limited, 0, sizeof(unsigned int) * c->np(), c->stream);
  (void)hipMemsetAsync(c->d_rate, 0, sizeof(unsigned long long) * c->np(), c->stream);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(sU);
  (void)hipFree(sdt);
  if (sB) (void)hipFree(sB);
  drop_graph(c);
  return rc != ADER_OK ? rc : rc2;
}

}  // namespace

extern "C" {

int ader_create(const ader_mesh* mesh, int system, int device, void* stream, ader_ctx** out) {
  return create(1, mesh, system, device, stream, out);
}

int ader_batch_create(int n, const ader_mesh* meshes, int system, int device, void* stream,
                      ader_ctx** out) {
  return create(n, meshes, system, device, stream, out);
}

int ader_batch_size(ader_ctx* c, int* n_out) {
  if (!c || !n_out) return ADER_EINVAL;
  *n_out = c->np();
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
  c->order = order;
  c->form = form;
  return ADER_OK;
}

int ader_set_riemann(ader_ctx* c, int riemann) {
  if (!c || (riemann != ADER_HLL && riemann != ADER_LINEARIZED)) return ADER_EINVAL;
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
  if (c->bounded) {
    long long ub = 0;
    for (const Problem& pr : c->probs) {
      if (!host_state_ok(U, nullptr, user_view(pr, ub), c->S_user, c->gamma)) return ADER_ESTATE;
      ub += (long long)pr.ux * pr.uy * pr.uz;
    }
    ADER_TRY(set_device(c));
    std::vector<double> hb;
    ub = 0;
    for (int q = 0; q < c->np(); ++q) {
      const Problem& pr = c->probs[q];
      hb.assign((size_t)5 * pr.N, 0.0);
      pack_interior(pr, U, c->S_user, ub, hb.data());
      ADER_TRY(put_problem(c, q, hb.data(), nullptr));
      ADER_TRY(check(hipStreamSynchronize(c->stream)));
      ub += (long long)pr.ux * pr.uy * pr.uz;
    }
    c->set_flags.assign(c->np(), 1);
    c->have_state = true;
    return ADER_OK;
  }
  for (const Problem& pr : c->probs)
    if (!host_state_ok(U, B, pr, c->S, c->gamma, c->system != ADER_LINADV)) return ADER_ESTATE;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipMemcpyAsync(c->U, U, sizeof(double) * 5 * (size_t)c->S, hipMemcpyHostToDevice,
                                c->stream)));
  if (mhd)
    ADER_TRY(check(hipMemcpyAsync(c->B, B, sizeof(double) * 3 * (size_t)c->S,
                                  hipMemcpyHostToDevice, c->stream)));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  c->set_flags.assign(c->np(), 1);
  c->have_state = true;
  return ADER_OK;
}

int ader_batch_set_state(ader_ctx* c, int i, const double* U, const double* B) {
  if (!c || !U || i < 0 || i >= c->np()) return ADER_EINVAL;
  const bool mhd = c->system == ADER_MHD;
  if (mhd != (B != nullptr)) return ADER_EINVAL;
  Problem lone = c->probs[i];
  lone.base = 0;
  if (c->bounded) {
    const Problem uv = user_view(lone, 0);
    if (!host_state_ok(U, nullptr, uv, uv.N, c->gamma)) return ADER_ESTATE;
    ADER_TRY(set_device(c));
    std::vector<double> hb((size_t)5 * lone.N, 0.0);
    pack_interior(lone, U, uv.N, 0, hb.data());
    ADER_TRY(put_problem(c, i, hb.data(), nullptr));
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
    c->set_flags[i] = 1;
    c->have_state = std::all_of(c->set_flags.begin(), c->set_flags.end(),
                                [](char f) { return f != 0; });
    return ADER_OK;
  }
  if (!host_state_ok(U, B, lone, lone.N, c->gamma, c->system != ADER_LINADV)) return ADER_ESTATE;
  ADER_TRY(set_device(c));
  ADER_TRY(put_problem(c, i, U, B));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  c->set_flags[i] = 1;
  c->have_state = std::all_of(c->set_flags.begin(), c->set_flags.end(), [](char f) { return f != 0; });
  return ADER_OK;
}

int ader_bind_device_state(ader_ctx* c, void* dU, void* dB) {
  if (!c || !dU) return ADER_EINVAL;
  if (c->bounded) return ADER_EUNSUPPORTED;   // the device layout holds ghost zones
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
  c->set_flags.assign(c->np(), 1);
  c->have_state = true;
  return ADER_OK;
}

int ader_get_state(ader_ctx* c, double* U, double* B) {
  if (!c || !U) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  if (c->bounded) {
    std::vector<double> hb;
    long long ub = 0;
    for (int q = 0; q < c->np(); ++q) {
      const Problem& pr = c->probs[q];
      hb.resize((size_t)5 * pr.N);
      ADER_TRY(get_problem(c, q, hb.data(), nullptr));
      unpack_interior(pr, hb.data(), U, c->S_user, ub);
      ub += (long long)pr.ux * pr.uy * pr.uz;
    }
    return ADER_OK;
  }
  ADER_TRY(check(hipMemcpyAsync(U, c->U, sizeof(double) * 5 * (size_t)c->S, hipMemcpyDeviceToHost,
                                c->stream)));
  if (B && c->system == ADER_MHD)
    ADER_TRY(check(hipMemcpyAsync(B, c->B, sizeof(double) * 3 * (size_t)c->S,
                                  hipMemcpyDeviceToHost, c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

int ader_batch_get_state(ader_ctx* c, int i, double* U, double* B) {
  if (!c || !U || i < 0 || i >= c->np()) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  if (c->bounded) {
    const Problem& pr = c->probs[i];
    std::vector<double> hb((size_t)5 * pr.N);
    ADER_TRY(get_problem(c, i, hb.data(), nullptr));
    unpack_interior(pr, hb.data(), U, (long long)pr.ux * pr.uy * pr.uz, 0);
    return ADER_OK;
  }
  return get_problem(c, i, U, B);
}

int ader_compute_dt(ader_ctx* c, double cfl, double* dt_out) {
  if (!c || !(cfl > 0.0) || !std::isfinite(cfl)) return ADER_EINVAL;
  if (dt_out && c->np() != 1) return ADER_EINVAL;
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
  ADER_TRY(ensure_work(c));
  k_set_dt<><<<(c->np() + 63) / 64, 64, 0, c->stream>>>(c->d_dt, c->np(), dt);
  ADER_TRY(launched());
  ADER_TRY(fill_ghosts(c));
  c->have_dt = true;
  return queue_step(c);
}

int ader_step_cfl(ader_ctx* c, double cfl) {
  if (!c || !(cfl > 0.0) || !std::isfinite(cfl)) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  return run_step_cfl(c, cfl);
}

int ader_batch_step_cfl(ader_ctx* c, double cfl, double* dts_out) {
  ADER_TRY(ader_step_cfl(c, cfl));
  if (!dts_out) return ADER_OK;
  ADER_TRY(read_status(c));
  ADER_TRY(check(hipMemcpyAsync(dts_out, c->d_dt, sizeof(double) * c->np(), hipMemcpyDeviceToHost,
                                c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

int ader_get_dt(ader_ctx* c, double* dt_out) {
  if (!c || !dt_out) return ADER_EINVAL;
  if (!c->have_dt) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipMemcpyAsync(dt_out, c->d_dt, sizeof(double) * c->np(), hipMemcpyDeviceToHost,
                                c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

int ader_synchronize(ader_ctx* c) {
  if (!c) return ADER_EINVAL;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  ADER_TRY(check(hipGetLastError()));
  return read_status(c);
}

int ader_set_graph(ader_ctx* c, int enable) {
  if (!c) return ADER_EINVAL;
  if (enable && c->stream == nullptr) return ADER_EUNSUPPORTED;
  ADER_TRY(set_device(c));
  if (!enable) {
    ADER_TRY(check(hipStreamSynchronize(c->stream)));
    drop_graph(c);
  }
  c->use_graph = enable != 0;
  return ADER_OK;
}

int ader_autotune(ader_ctx* c, int reps) {
  if (!c || reps < 1 || reps > 1000) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  return autotune(c, reps);
}

int ader_get_launch(ader_ctx* c, int* block_out, int* blocks_per_cu_out) {
  if (!c || !block_out || !blocks_per_cu_out) return ADER_EINVAL;
  for (int q = 0; q < kNumClasses; ++q) {
    block_out[q] = c->shape[q].block;
    blocks_per_cu_out[q] = c->shape[q].blocks_per_cu;
  }
  return ADER_OK;
}

int ader_set_launch(ader_ctx* c, const int* block, const int* blocks_per_cu) {
  if (!c || !block || !blocks_per_cu) return ADER_EINVAL;
  for (int q = 0; q < kNumClasses; ++q)
    if (block[q] < 64 || block[q] > 256 || block[q] % 64 != 0 || blocks_per_cu[q] < 1 ||
        blocks_per_cu[q] > 64)
      return ADER_EINVAL;
  for (int q = 0; q < kNumClasses; ++q) c->shape[q] = LaunchShape{block[q], blocks_per_cu[q]};
  return ADER_OK;
}

int ader_set_layout(ader_ctx* c, int layout) {
  if (!c || layout < -1 || layout >= kNumLayouts) return ADER_EINVAL;
  if ((layout == ADER_LAYOUT_SPLIT || layout == ADER_LAYOUT_SPLIT2) && c->order < 3)
    return ADER_EUNSUPPORTED;
  if (layout == ADER_LAYOUT_ZONE2 && c->order > 3) return ADER_EUNSUPPORTED;
  if (layout == ADER_LAYOUT_ZONE_2W && (c->order > 3 || c->system == ADER_MHD))
    return ADER_EUNSUPPORTED;
  if ((layout == ADER_LAYOUT_PAIR || layout == ADER_LAYOUT_PAIR2 ||
       layout == ADER_LAYOUT_PAIR_SPLIT) &&
      (c->order < 3 || c->system != ADER_MHD))
    return ADER_EUNSUPPORTED;
  if ((layout == ADER_LAYOUT_PAIR || layout == ADER_LAYOUT_PAIR2) && c->order == 4)
    return ADER_EUNSUPPORTED;
  if (layout == ADER_LAYOUT_FUSED && (c->order != 3 || c->system != ADER_EULER))
    return ADER_EUNSUPPORTED;
  // Euler in FP64 at order 4 runs the lane-split predictor only
  if (layout == ADER_LAYOUT_ZONE && c->order == 4 && c->system == ADER_EULER &&
      c->precision == ADER_FP64)
    return ADER_EUNSUPPORTED;
  c->layout = layout;
  return ADER_OK;
}

int ader_set_scheme(ader_ctx* c, int scheme) {
  if (!c || (scheme != ADER_SCHEME_ADER && scheme != ADER_SCHEME_SSPRK)) return ADER_EINVAL;
  c->scheme = scheme;
  return ADER_OK;
}

int ader_get_scheme(ader_ctx* c, int* scheme_out) {
  if (!c || !scheme_out) return ADER_EINVAL;
  *scheme_out = c->scheme;
  return ADER_OK;
}

int ader_set_positivity(ader_ctx* c, int mode) {
  if (!c || (mode != ADER_POSITIVITY_CHECK && mode != ADER_POSITIVITY_LIMIT)) return ADER_EINVAL;
  c->positivity = mode;
  return ADER_OK;
}

int ader_set_advection(ader_ctx* c, double ax, double ay, double az) {
  if (!c) return ADER_EINVAL;
  if (c->system != ADER_LINADV) return ADER_EUNSUPPORTED;
  if (!std::isfinite(ax) || !std::isfinite(ay) || !std::isfinite(az)) return ADER_EINVAL;
  if (ax == 0.0 && ay == 0.0 && az == 0.0) return ADER_EINVAL;
  c->adv[0] = ax;
  c->adv[1] = ay;
  c->adv[2] = az;
  return ADER_OK;
}

int ader_set_boundary(ader_ctx* c, const int* bc) {
  if (!c || !bc) return ADER_EINVAL;
  for (int f = 0; f < 6; ++f)
    if (bc[f] != ADER_BC_PERIODIC && bc[f] != ADER_BC_OUTFLOW && bc[f] != ADER_BC_REFLECT &&
        bc[f] != ADER_BC_INFLOW)
      return ADER_EINVAL;
  for (int a = 0; a < 3; ++a)
    if ((bc[2 * a] == ADER_BC_PERIODIC) != (bc[2 * a + 1] == ADER_BC_PERIODIC)) return ADER_EINVAL;
  if (c->system != ADER_EULER) return ADER_EUNSUPPORTED;
  if (c->bounded || !c->owns_U ||
      std::any_of(c->set_flags.begin(), c->set_flags.end(), [](char f) { return f != 0; }))
    return ADER_ESEQ;
  const bool bnd[3] = {bc[0] != ADER_BC_PERIODIC, bc[2] != ADER_BC_PERIODIC,
                       bc[4] != ADER_BC_PERIODIC};
  if (!bnd[0] && !bnd[1] && !bnd[2]) return ADER_OK;
  // the padded meshes: kGhost layers on each bounded face, the zone size kept
  std::vector<ader_mesh> meshes;
  for (const Problem& pr : c->probs) {
    if ((bnd[0] && pr.ux < kGhost) || (bnd[1] && pr.uy < kGhost) || (bnd[2] && pr.uz < kGhost))
      return ADER_EINVAL;
    ader_mesh m;
    m.nx = pr.ux + (bnd[0] ? 2 * kGhost : 0);
    m.ny = pr.uy + (bnd[1] ? 2 * kGhost : 0);
    m.nz = pr.uz + (bnd[2] ? 2 * kGhost : 0);
    m.lx = pr.dx * m.nx;
    m.ly = pr.dy * m.ny;
    m.lz = pr.dz * m.nz;
    meshes.push_back(m);
  }
  ADER_TRY(set_device(c));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  ader_ctx* t = nullptr;
  ADER_TRY(create(c->np(), meshes.data(), c->system, c->device, c->stream, &t));
  for (int q = 0; q < t->np(); ++q) {
    Problem& pr = t->probs[q];
    pr.ux = c->probs[q].ux;
    pr.uy = c->probs[q].uy;
    pr.uz = c->probs[q].uz;
    pr.dx = c->probs[q].dx;
    pr.dy = c->probs[q].dy;
    pr.dz = c->probs[q].dz;
    pr.gx = bnd[0] ? kGhost : 0;
    pr.gy = bnd[1] ? kGhost : 0;
    pr.gz = bnd[2] ? kGhost : 0;
    for (int f = 0; f < 6; ++f) pr.bc[f] = bc[f];
  }
  if (hipMemcpy(t->d_probs, t->probs.data(), sizeof(Problem) * t->probs.size(),
                hipMemcpyHostToDevice) != hipSuccess) {
    ader_destroy(t);
    return ADER_EDEVICE;
  }
  // the settings carry over; the new layout's buffers replace the old ones
  t->gamma = c->gamma;
  t->order = c->order;
  t->form = c->form;
  t->riemann = c->riemann;
  t->precision = c->precision;
  t->positivity = c->positivity;
  t->layout = c->layout;
  t->recon_mode = c->recon_mode;
  t->flux_mode = c->flux_mode;
  t->scheme = c->scheme;
  t->use_graph = c->use_graph;
  for (int q = 0; q < kNumClasses; ++q) t->shape[q] = c->shape[q];
  t->has_source = c->has_source;
  t->source = c->source;
  t->source_version = c->source_version;
  t->bounded = true;
  t->S_user = c->S_user;
  t->inflow = c->inflow;
  t->inflow_set = c->inflow_set;
  t->inflow_version = c->inflow_version;
  std::swap(*c, *t);
  ader_destroy(t);
  return ADER_OK;
}

int ader_set_inflow(ader_ctx* c, int face, const double* state) {
  if (!c || !state || face < 0 || face >= 6) return ADER_EINVAL;
  if (c->system != ADER_EULER) return ADER_EUNSUPPORTED;
  for (int v = 0; v < 5; ++v)
    if (!std::isfinite(state[v])) return ADER_EINVAL;
  const double r = state[0];
  const double p = (c->gamma - 1.0) * (state[4] - 0.5 * (state[1] * state[1] + state[2] * state[2] +
                                                         state[3] * state[3]) / r);
  if (!(r > 0.0) || !(p > 0.0)) return ADER_EINVAL;
  for (int v = 0; v < 5; ++v) c->inflow.v[face][v] = state[v];
  c->inflow_set |= 1u << face;
  ++c->inflow_version;
  return ADER_OK;
}

int ader_set_source(ader_ctx* c, const double* A, const double* b) {
  if (!c) return ADER_EINVAL;
  if (c->system != ADER_EULER) return ADER_EUNSUPPORTED;
  if (!A) {
    if (b) return ADER_EINVAL;
    c->has_source = false;
    c->source = SourceAffine{};
    ++c->source_version;
    return ADER_OK;
  }
  SourceAffine s{};
  for (int q = 0; q < 25; ++q) {
    if (!std::isfinite(A[q])) return ADER_EINVAL;
    s.A[q] = A[q];
  }
  for (int v = 0; v < 5; ++v) {
    const double bv = b ? b[v] : 0.0;
    if (!std::isfinite(bv)) return ADER_EINVAL;
    s.b[v] = bv;
  }
  c->source = s;
  c->has_source = true;
  ++c->source_version;
  return ADER_OK;
}

int ader_get_positivity(ader_ctx* c, int* mode_out) {
  if (!c || !mode_out) return ADER_EINVAL;
  *mode_out = c->positivity;
  return ADER_OK;
}

int ader_limited_zones(ader_ctx* c, long long* counts_out) {
  if (!c || !counts_out) return ADER_EINVAL;
  ADER_TRY(set_device(c));
  std::vector<unsigned int> cnt(c->np(), 0u);
  ADER_TRY(check(hipMemcpyAsync(cnt.data(), c->d_limited, sizeof(unsigned int) * cnt.size(),
                                hipMemcpyDeviceToHost, c->stream)));
  ADER_TRY(check(hipMemsetAsync(c->d_limited, 0, sizeof(unsigned int) * cnt.size(), c->stream)));
  ADER_TRY(check(hipStreamSynchronize(c->stream)));
  for (int q = 0; q < c->np(); ++q) counts_out[q] = (long long)cnt[q];
  return ADER_OK;
}

int ader_set_recon(ader_ctx* c, int mode) {
  if (!c || (mode != -1 && mode != ADER_RECON_SWEEPS && mode != ADER_RECON_TILED &&
             mode != ADER_RECON_COLUMNS && mode != ADER_RECON_MARCH))
    return ADER_EINVAL;
  c->recon_mode = mode;
  return ADER_OK;
}

int ader_get_recon(ader_ctx* c, int* mode_out) {
  if (!c || !mode_out) return ADER_EINVAL;
  *mode_out = (c->order >= 3 && c->recon_mode >= 0) ? c->recon_mode : ADER_RECON_SWEEPS;
  return ADER_OK;
}

int ader_set_flux_mode(ader_ctx* c, int mode) {
  if (!c || (mode != -1 && mode != ADER_FLUX_SEPARATE && mode != ADER_FLUX_FUSED))
    return ADER_EINVAL;
  if (mode == ADER_FLUX_FUSED && c->system != ADER_EULER) return ADER_EUNSUPPORTED;
  c->flux_mode = mode;
  return ADER_OK;
}

int ader_get_flux_mode(ader_ctx* c, int* mode_out) {
  if (!c || !mode_out) return ADER_EINVAL;
  *mode_out = c->flux_fused() ? ADER_FLUX_FUSED : ADER_FLUX_SEPARATE;
  return ADER_OK;
}

int ader_get_layout(ader_ctx* c, int* layout_out) {
  if (!c || !layout_out) return ADER_EINVAL;
  const StageFns* s = stages_of(c);
  *layout_out = s ? layout_of(c, s) : (c->layout < 0 ? ADER_LAYOUT_ZONE : c->layout);
  return ADER_OK;
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
    case ADER_EUNSUPPORTED: return "not supported";
    case ADER_ENOMEM: return "device allocation failed";
    case ADER_EDEVICE: return "HIP runtime error";
    case ADER_ESTATE:
      return "unphysical state (rho <= 0, P <= 0 or non-finite, in a zone or at a check point)";
    case ADER_ESEQ: return "call out of sequence";
  }
  return "unknown error";
}

void ader_destroy(ader_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  drop_events(c);
  free_buffers(c);
  delete c;
}

}  // extern "C"
