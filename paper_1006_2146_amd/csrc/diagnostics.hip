// Conserved totals and the largest discrete divergence of the face field,
// per problem of a context, on the device: the properties the step keeps by
// construction -- eq. (6) changes the totals only by face fluxes, which
// cancel on a periodic mesh, and the constrained transport of eq. (8) keeps
// the divergence of the face field at its initial round-off level.
//
// Reductions are deterministic: every problem is cut into tiles of a fixed
// number of zones; one block of a fixed 256 threads reduces a tile in a fixed
// order (strided per-thread sums, then a fixed tree in LDS) into a partial
// row, and a second kernel reduces each problem's partial rows the same way.
// No atomics take part, so the result depends neither on the launch shape
// nor on timing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ader_ctx.h"
#include "recon_tile.h"

namespace ader {
namespace {

constexpr int kDiagThreads = 256;

// Per zone: the five hydro variables, the three face-field components and
// |div B| (lower faces of the zone and of its upper neighbours; eq. 8's
// discrete divergence, differences per axis summed in x, y, z order).
__device__ __forceinline__ void diag_zone(const double* __restrict__ U,
                                          const double* __restrict__ B, const Grid& g,
                                          const Problem& pr, long long n, double (&acc)[kDiagVals]) {
  if (pr.gx | pr.gy | pr.gz) {   // bounded problem: its interior only
    int i, j, k;
    zone_ijk(g, n, i, j, k);
    if (ghost_zone(pr, i, j, k)) return;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) acc[v] += U[(long long)v * g.S + n];
  if (!B) return;
  int i, j, k;
  zone_ijk(g, n, i, j, k);
  const long long up[3] = {zone_of(wrap(i + 1, g.nx), j, k, g), zone_of(i, wrap(j + 1, g.ny), k, g),
                           zone_of(i, j, wrap(k + 1, g.nz), g)};
  const double dx[3] = {pr.dx, pr.dy, pr.dz};
  double div = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double lo = B[(long long)d * g.S + n];
    acc[5 + d] += lo;
    div += (B[(long long)d * g.S + up[d]] - lo) / dx[d];
  }
  acc[8] = fmax(acc[8], fabs(div));
}

// Fixed-order tree over the block's 256 rows of LDS (sums; the last value a
// max); the block's result ends in row 0.
__device__ __forceinline__ void block_tree(double (*s)[kDiagVals]) {
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < kDiagVals - 1; ++v) s[threadIdx.x][v] += s[threadIdx.x + w][v];
      s[threadIdx.x][kDiagVals - 1] =
          fmax(s[threadIdx.x][kDiagVals - 1], s[threadIdx.x + w][kDiagVals - 1]);
    }
  }
  __syncthreads();
}

// One block per tile (block-strided over the tiles): partial[t][v].
template <int = 0>
__global__ void __launch_bounds__(kDiagThreads) k_diag_tiles(const double* __restrict__ U,
                                                             const double* __restrict__ B, Batch b,
                                                             const long long* __restrict__ tile_base,
                                                             double* __restrict__ partial) {
  __shared__ double s[kDiagThreads][kDiagVals];
  const long long ntiles = tile_base[b.np];
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int p = problem_of_tile(tile_base, b.np, t);
    const Problem pr = b.P[p];
    const Grid g{pr.nx, pr.ny, pr.nz, pr.N, b.S, pr.base};
    const long long lo = pr.base + (t - tile_base[p]) * kDiagTile;
    const long long hi = lo + kDiagTile < pr.base + pr.N ? lo + kDiagTile : pr.base + pr.N;
    double acc[kDiagVals] = {};
    for (long long n = lo + threadIdx.x; n < hi; n += kDiagThreads) diag_zone(U, B, g, pr, n, acc);
#pragma unroll
    for (int v = 0; v < kDiagVals; ++v) s[threadIdx.x][v] = acc[v];
    block_tree(s);
    if (threadIdx.x == 0)
#pragma unroll
      for (int v = 0; v < kDiagVals; ++v) partial[t * kDiagVals + v] = s[0][v];
    __syncthreads();
  }
}

// One block per problem: its tiles' partial rows in the same fixed order;
// totals[p][v] = the sum times the zone volume (v < 8), maxdiv[p].
template <int = 0>
__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ partial,
                                                             Batch b,
                                                             const long long* __restrict__ tile_base,
                                                             double* __restrict__ totals,
                                                             double* __restrict__ maxdiv) {
  __shared__ double s[kDiagThreads][kDiagVals];
  const int p = blockIdx.x;
  double acc[kDiagVals] = {};
  for (long long t = tile_base[p] + threadIdx.x; t < tile_base[p + 1]; t += kDiagThreads) {
#pragma unroll
    for (int v = 0; v < kDiagVals - 1; ++v) acc[v] += partial[t * kDiagVals + v];
    acc[kDiagVals - 1] = fmax(acc[kDiagVals - 1], partial[t * kDiagVals + kDiagVals - 1]);
  }
#pragma unroll
  for (int v = 0; v < kDiagVals; ++v) s[threadIdx.x][v] = acc[v];
  block_tree(s);
  if (threadIdx.x == 0) {
    const Problem pr = b.P[p];
    const double vol = pr.dx * pr.dy * pr.dz;   // (a padded problem keeps the zone size)
#pragma unroll
    for (int v = 0; v < kDiagVals - 1; ++v) totals[p * (kDiagVals - 1) + v] = s[0][v] * vol;
    maxdiv[p] = s[0][kDiagVals - 1];
  }
}

}  // namespace

// Queues both passes with the given device scratch (partial: ntiles rows of
// kDiagVals; totals: np rows of 8; maxdiv: np) and copies the results to the
// caller's host arrays (either may be null), synchronising the stream.
int diagnostics_into(ader_ctx* c, double* partial, double* d_totals, double* d_maxdiv,
                     double* totals, double* maxdiv) {
  const Batch b = c->batch();
  const long long cap = 8LL * c->num_cus;
  const unsigned g = (unsigned)(c->ndiag_tiles < cap ? c->ndiag_tiles : cap);
  k_diag_tiles<><<<g < 1 ? 1 : g, kDiagThreads, 0, c->stream>>>(
      c->U, c->system == ADER_MHD ? c->B : nullptr, b, c->d_diag_base, partial);
  ADER_TRY(launched());
  k_diag_final<><<<c->np(), kDiagThreads, 0, c->stream>>>(partial, b, c->d_diag_base, d_totals,
                                                          d_maxdiv);
  ADER_TRY(launched());
  if (totals)
    ADER_TRY(check(hipMemcpyAsync(totals, d_totals, sizeof(double) * (kDiagVals - 1) * c->np(),
                                  hipMemcpyDeviceToHost, c->stream)));
  if (maxdiv)
    ADER_TRY(check(hipMemcpyAsync(maxdiv, d_maxdiv, sizeof(double) * c->np(),
                                  hipMemcpyDeviceToHost, c->stream)));
  return check(hipStreamSynchronize(c->stream));
}

// Scratch of ader_diagnostics_noalloc: the partial rows of at most
// kStaticTiles tiles (134 M zones in tiles of 8192) and the results of at
// most kStaticProblems problems, 1.47 MB on every device the library runs
// this entry point on, held until the process ends.  Host code never passes
// `scratch` itself to a kernel or a copy: it stands in for the device copy
// only on the device side; its device address comes from
// hipGetSymbolAddress, per device.
constexpr long long kStaticTiles = 16384;
constexpr int kStaticProblems = 4096;
static __device__ __align__(256) double
    scratch[(kStaticTiles + kStaticProblems) * kDiagVals];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of `scratch` on `device` (which must be current),
// looked up once per device.
int static_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return ADER_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return ADER_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return ADER_OK;
}

}  // namespace ader

using namespace ader;

extern "C" int ader_diagnostics(ader_ctx* c, double* totals, double* max_abs_divB) {
  if (!c) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(check(hipSetDevice(c->device)));
  if (!c->d_diag) {
    const size_t bytes =
        sizeof(double) * ((size_t)c->ndiag_tiles * kDiagVals + (size_t)c->np() * kDiagVals);
    if (hipMalloc(&c->d_diag, bytes) != hipSuccess) {
      c->d_diag = nullptr;
      (void)hipGetLastError();
      return ADER_ENOMEM;
    }
    c->fixed_bytes += bytes;
    c->bytes += bytes;
  }
  double* d_tot = c->d_diag + (size_t)c->ndiag_tiles * kDiagVals;
  return diagnostics_into(c, c->d_diag, d_tot, d_tot + (size_t)c->np() * (kDiagVals - 1), totals,
                          max_abs_divB);
}

extern "C" int ader_diagnostics_noalloc(ader_ctx* c, double* totals, double* max_abs_divB) {
  if (!c) return ADER_EINVAL;
  if (c->ndiag_tiles > kStaticTiles || c->np() > kStaticProblems) return ADER_EINVAL;
  if (!c->have_state) return ADER_ESEQ;
  ADER_TRY(check(hipSetDevice(c->device)));
  double* p = nullptr;
  ADER_TRY(static_scratch(c->device, &p));
  // every partial row and result is written before it is read: nothing to
  // clear between calls
  double* d_tot = p + (size_t)kStaticTiles * kDiagVals;
  return diagnostics_into(c, p, d_tot, d_tot + (size_t)kStaticProblems * (kDiagVals - 1), totals,
                          max_abs_divB);
}
