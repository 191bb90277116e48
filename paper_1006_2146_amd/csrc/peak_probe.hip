// Peak probes: the vector FMA rate this library's code can reach (FP32 as
// compiled here, without packed FP32 instructions, and FP64) and the HBM
// copy bandwidth, each timed with HIP events on a stream of its own.  They
// are the measured denominators of the step kernels' rooflines.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/ader.h"
#include "../../include/ader_probe.h"
#include "generated/face_rows.h"

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

// ---------------------------------------------------------------------------
// VALU against MFMA on the face-point evaluation of the predictor: for each
// zone and each of 5 variables, the values of the space-time polynomial at
// the P side points from its K modes, y = R x, then the sum of y^2 over the
// points and variables (one number per zone, so both engines consume every
// product the same way).  Variable v takes the modes x + v.
// ---------------------------------------------------------------------------
template <int ORDER>
struct FaceRows;
template <>
struct FaceRows<3> {
  static constexpr int P = ader_gen::kFaceP3, K = ader_gen::kFaceK3, NNZ = ader_gen::kFaceNnz3;
  __host__ __device__ static constexpr float at(int p, int k) { return ader_gen::kFaceRows3[p][k]; }
};
template <>
struct FaceRows<4> {
  static constexpr int P = ader_gen::kFaceP4, K = ader_gen::kFaceK4, NNZ = ader_gen::kFaceNnz4;
  __host__ __device__ static constexpr float at(int p, int k) { return ader_gen::kFaceRows4[p][k]; }
};

constexpr int kFaceVars = 5;

// one lane per zone, the matrix's nonzero entries as immediate operands (the
// form the predictor kernels take): NNZ multiply-adds per variable
template <int ORDER>
__global__ __launch_bounds__(kBlock) void k_face_valu(const float* __restrict__ X,
                                                      float* __restrict__ out, int nz) {
  using R = FaceRows<ORDER>;
  for (int z = blockIdx.x * kBlock + threadIdx.x; z < nz; z += gridDim.x * kBlock) {
    float x[R::K];
#pragma unroll
    for (int k = 0; k < R::K; ++k) x[k] = X[(size_t)k * nz + z];
    float sum = 0.f;
#pragma unroll
    for (int v = 0; v < kFaceVars; ++v) {
      float xv[R::K];
#pragma unroll
      for (int k = 0; k < R::K; ++k) xv[k] = x[k] + float(v);
#pragma unroll
      for (int p = 0; p < R::P; ++p) {
        float y = 0.f;
#pragma unroll
        for (int k = 0; k < R::K; ++k) {
          if (R::at(p, k) != 0.f) y = fmaf(R::at(p, k), xv[k], y);   // folded at compile time
        }
        sum = fmaf(y, y, sum);
      }
    }
    out[z] = sum;
  }
}

// 32 zones per wave through v_mfma_f32_32x32x2f32: D (32 points x 32 zones)
// = A (32 points x 2 modes, the matrix) B (2 modes x 32 zones), K/2 steps per
// 32-point tile, the matrix zero-padded to whole tiles and an even mode
// count.  Lane l: A holds R[32 t + l % 32][2 s + l / 32], B the mode
// 2 s + l / 32 of zone l % 32, and D the zone l % 32's values at 16 of the
// tile's points; the two halves of the wave add their partial sums.  Rm is
// the matrix, row-major P x K, in device memory.
template <int ORDER>
__global__ __launch_bounds__(kBlock) void k_face_mfma(const float* __restrict__ X,
                                                      const float* __restrict__ Rm,
                                                      float* __restrict__ out, int nz) {
  using R = FaceRows<ORDER>;
  constexpr int PT = (R::P + 31) / 32, KS = (R::K + 1) / 2;
  typedef float f16v __attribute__((ext_vector_type(16)));
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  float a[PT][KS];
#pragma unroll
  for (int t = 0; t < PT; ++t)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int p = 32 * t + c, k = 2 * s + h;
      a[t][s] = (p < R::P && k < R::K) ? Rm[p * R::K + k] : 0.f;
    }
  const int waves = gridDim.x * (kBlock / 64);
  for (int g = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); g * 32 < nz; g += waves) {
    const int z = g * 32 + c;
    const bool in = z < nz;
    float xb[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 2 * s + h;
      xb[s] = (in && k < R::K) ? X[(size_t)k * nz + z] : 0.f;
    }
    float sum = 0.f;
#pragma unroll
    for (int v = 0; v < kFaceVars; ++v) {
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        f16v acc = {};
#pragma unroll
        for (int s = 0; s < KS; ++s)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t][s], xb[s] + float(v), acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; ++r) sum = fmaf(acc[r], acc[r], sum);
      }
    }
    sum += __shfl_xor(sum, 32);
    if (h == 0 && in) out[z] = sum;
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


// device current, its compute units, the probe's stream and events
int open_probe(int device, Probe& p, int* cus) {
  int ndev = 0;
  PROBE_TRY(ok(hipGetDeviceCount(&ndev)));
  if (device < 0 || device >= ndev) return ADER_EINVAL;
  PROBE_TRY(ok(hipSetDevice(device)));
  PROBE_TRY(ok(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, device)));
  PROBE_TRY(ok(hipStreamCreate(&p.s)));
  PROBE_TRY(ok(hipEventCreate(&p.e0)));
  PROBE_TRY(ok(hipEventCreate(&p.e1)));
  return ADER_OK;
}

// x[i] in [-1, 1) from a hash of i
__global__ __launch_bounds__(kBlock) void k_fill_probe(float* __restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kBlock) {
    unsigned h = (unsigned)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = float(h >> 8) * (2.0f / 16777216.0f) - 1.0f;
  }
}

template <int ORDER>
int face_eval(Probe& p, int cus, double* out) {
  using R = FaceRows<ORDER>;
  constexpr int PT = (R::P + 31) / 32, KS = (R::K + 1) / 2;
  const int nz = 1 << 22;
  float *X = nullptr, *Rm = nullptr, *ov = nullptr, *om = nullptr;
  const size_t nx = (size_t)R::K * nz;
  if (hipMalloc(&p.a, sizeof(float) * nx) != hipSuccess ||
      hipMalloc(&p.b, sizeof(float) * (2 * (size_t)nz + R::P * R::K)) != hipSuccess) {
    (void)hipGetLastError();
    return ADER_ENOMEM;
  }
  X = static_cast<float*>(p.a);
  ov = static_cast<float*>(p.b);
  om = ov + nz;
  Rm = om + nz;
  std::vector<float> rows(R::P * R::K);
  for (int q = 0; q < R::P; ++q)
    for (int k = 0; k < R::K; ++k) rows[q * R::K + k] = R::at(q, k);
  PROBE_TRY(ok(hipMemcpyAsync(Rm, rows.data(), sizeof(float) * rows.size(),
                              hipMemcpyHostToDevice, p.s)));
  const unsigned grid = (unsigned)cus * 8u;
  k_fill_probe<<<grid, kBlock, 0, p.s>>>(X, nx);
  PROBE_TRY(ok(hipGetLastError()));
  double tv = 0.0, tm = 0.0;
  PROBE_TRY(best_ms(p, 5, [&] { k_face_valu<ORDER><<<grid, kBlock, 0, p.s>>>(X, ov, nz); }, &tv));
  PROBE_TRY(best_ms(p, 5, [&] {
    k_face_mfma<ORDER><<<grid, kBlock, 0, p.s>>>(X, Rm, om, nz);
  }, &tm));
  std::vector<float> a(nz), b(nz);
  PROBE_TRY(ok(hipMemcpyAsync(a.data(), ov, sizeof(float) * nz, hipMemcpyDeviceToHost, p.s)));
  PROBE_TRY(ok(hipMemcpyAsync(b.data(), om, sizeof(float) * nz, hipMemcpyDeviceToHost, p.s)));
  PROBE_TRY(ok(hipStreamSynchronize(p.s)));
  double diff = 0.0;
  for (int z = 0; z < nz; ++z) {
    const double d = std::fabs((double)a[z] - (double)b[z]) / std::fmax(std::fabs((double)a[z]), 1e-30);
    diff = d > diff ? d : diff;
  }
  const double useful = 2.0 * R::NNZ * kFaceVars * (double)nz;
  const double dense = 2.0 * (32.0 * PT) * (2.0 * KS) * kFaceVars * (double)nz;
  out[0] = useful / (tv * 1e-3) / 1e12;
  out[1] = useful / (tm * 1e-3) / 1e12;
  out[2] = tv;
  out[3] = tm;
  out[4] = dense / (tm * 1e-3) / 1e12;
  out[5] = diff;
  return ADER_OK;
}

}  // namespace

extern "C" int ader_probe_face_eval(int device, int order, double* out) {
  if (!out || (order != 3 && order != 4)) return ADER_EINVAL;
  Probe p;
  int cus = 0;
  PROBE_TRY(open_probe(device, p, &cus));
  return order == 3 ? face_eval<3>(p, cus, out) : face_eval<4>(p, cus, out);
}

extern "C" int ader_probe_peak(int device, int kind, double* value_out) {
  if (!value_out || kind < ADER_PROBE_FP32_FMA || kind > ADER_PROBE_HBM_COPY) return ADER_EINVAL;
  Probe p;
  int cus = 0;
  PROBE_TRY(open_probe(device, p, &cus));
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
