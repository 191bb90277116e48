// Peak probes: the vector FMA rate this library's code can reach (FP32 as
// compiled here, without packed FP32 instructions, and FP64) and the HBM
// copy bandwidth, each timed with HIP events on a stream of its own.  They
// are the measured denominators of the step kernels' rooflines.
#include <hip/hip_runtime.h>

#include "../../include/ader.h"
#include "../../include/ader_probe.h"

namespace {

constexpr int kChains = 8;    // independent FMA chains per thread
constexpr int kUnroll = 16;   // FMAs per chain per loop trip
constexpr int kTrips = 2048;
constexpr int kBlock = 256;

// a <- a b + c on kChains independent chains; b < 1 and c > 0 keep every
// chain bounded and normal.  The store is taken only if the sum equals a
// value no chain can reach, so the stores cost nothing but keep the FMAs.
template <class T>
__global__ __launch_bounds__(kBlock) void k_fma_probe(T* __restrict__ out, T b, T c, T never) {
  T a[kChains];
#pragma unroll
  for (int q = 0; q < kChains; ++q) a[q] = T(threadIdx.x & 7) * T(0.125) + T(q);
#pragma unroll 1
  for (int t = 0; t < kTrips; ++t) {
#pragma unroll
    for (int r = 0; r < kUnroll; ++r)
#pragma unroll
      for (int q = 0; q < kChains; ++q) a[q] = fma(a[q], b, c);
  }
  T s = T(0);
#pragma unroll
  for (int q = 0; q < kChains; ++q) s += a[q];
  if (s == never) out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// Grid-stride copy of n float4 values, UNROLL loads in flight per thread
// before their stores (n a multiple of UNROLL x the grid's threads).
template <int UNROLL>
__global__ __launch_bounds__(kBlock) void k_copy_probe(const float4* __restrict__ src,
                                                       float4* __restrict__ dst, size_t n) {
  const size_t threads = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += threads * UNROLL) {
    float4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = src[i + u * threads];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) dst[i + u * threads] = v[u];
  }
}

struct Probe {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* a = nullptr;
  void* b = nullptr;
  ~Probe() {
    if (s) (void)hipStreamSynchronize(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  }
};

int ok(hipError_t e) { return e == hipSuccess ? ADER_OK : ADER_EDEVICE; }

#define PROBE_TRY(expr)             \
  do {                              \
    int _rc = (expr);               \
    if (_rc != ADER_OK) return _rc; \
  } while (0)

// Best of `reps` timed launches after one warm-up, in milliseconds.
template <class F>
int best_ms(Probe& p, int reps, F launch, double* ms) {
  launch();
  PROBE_TRY(ok(hipGetLastError()));
  double best = 1e30;
  for (int r = 0; r < reps; ++r) {
    PROBE_TRY(ok(hipEventRecord(p.e0, p.s)));
    launch();
    PROBE_TRY(ok(hipGetLastError()));
    PROBE_TRY(ok(hipEventRecord(p.e1, p.s)));
    PROBE_TRY(ok(hipEventSynchronize(p.e1)));
    float t = 0.f;
    PROBE_TRY(ok(hipEventElapsedTime(&t, p.e0, p.e1)));
    if (t < best) best = t;
  }
  *ms = best;
  return ADER_OK;
}

}  // namespace

extern "C" int ader_probe_peak(int device, int kind, double* value_out) {
  if (!value_out || kind < ADER_PROBE_FP32_FMA || kind > ADER_PROBE_HBM_COPY) return ADER_EINVAL;
  int ndev = 0;
  PROBE_TRY(ok(hipGetDeviceCount(&ndev)));
  if (device < 0 || device >= ndev) return ADER_EINVAL;
  PROBE_TRY(ok(hipSetDevice(device)));
  int cus = 0;
  PROBE_TRY(ok(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)));
  Probe p;
  PROBE_TRY(ok(hipStreamCreate(&p.s)));
  PROBE_TRY(ok(hipEventCreate(&p.e0)));
  PROBE_TRY(ok(hipEventCreate(&p.e1)));
  double ms = 0.0;
  if (kind == ADER_PROBE_HBM_COPY) {
    const size_t bytes = size_t(1) << 30;   // 1 GiB each way
    const size_t n = bytes / sizeof(float4);
    if (hipMalloc(&p.a, bytes) != hipSuccess || hipMalloc(&p.b, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return ADER_ENOMEM;
    }
    PROBE_TRY(ok(hipMemsetAsync(p.a, 0, bytes, p.s)));
    // the best over a few grid sizes and loads in flight; a grid whose
    // thread count times 4 does not divide n is skipped, so the unrolled
    // copy stays in bounds
    double best = 1e30;
    for (unsigned per_cu : {4u, 8u, 16u, 32u}) {
      const unsigned grid = (unsigned)cus * per_cu;
      if (n % ((size_t)grid * kBlock * 4) != 0) continue;
      double t1 = 0.0, t4 = 0.0;
      PROBE_TRY(best_ms(p, 5, [&] {
        k_copy_probe<1><<<grid, kBlock, 0, p.s>>>((const float4*)p.a, (float4*)p.b, n);
      }, &t1));
      PROBE_TRY(best_ms(p, 5, [&] {
        k_copy_probe<4><<<grid, kBlock, 0, p.s>>>((const float4*)p.a, (float4*)p.b, n);
      }, &t4));
      best = t1 < best ? t1 : best;
      best = t4 < best ? t4 : best;
    }
    if (best >= 1e30) return ADER_EINVAL;
    *value_out = 2.0 * (double)bytes / (best * 1e-3) / 1e9;   // GB/s, read + write
    return ADER_OK;
  }
  // 32 waves per CU (8 per SIMD) of FMA chains
  const unsigned grid = (unsigned)cus * 8u;
  const size_t threads = (size_t)grid * kBlock;
  const double flops = 2.0 * kChains * kUnroll * (double)kTrips * (double)threads;
  if (kind == ADER_PROBE_FP32_FMA) {
    if (hipMalloc(&p.a, threads * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return ADER_ENOMEM;
    }
    PROBE_TRY(best_ms(p, 5, [&] {
      k_fma_probe<float><<<grid, kBlock, 0, p.s>>>((float*)p.a, 0.999f, 0.001f, -1.0f);
    }, &ms));
  } else {
    if (hipMalloc(&p.a, threads * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return ADER_ENOMEM;
    }
    PROBE_TRY(best_ms(p, 5, [&] {
      k_fma_probe<double><<<grid, kBlock, 0, p.s>>>((double*)p.a, 0.999, 0.001, -1.0);
    }, &ms));
  }
  *value_out = flops / (ms * 1e-3) / 1e12;   // TFLOP/s
  return ADER_OK;
}
