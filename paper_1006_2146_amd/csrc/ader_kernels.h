// HIP kernels of one ADER-CG step (gfx950).  Every kernel is persistent over
// all zones of all problems of a batch (a lone problem is a batch of one):
// each thread walks zones of its block's contiguous chunk and applies the
// per-zone operation of zone_ops.h with the problem the zone belongs to.
#pragma once
#include <hip/hip_runtime.h>

#include "ader_ctx.h"
#include "lane_split.h"
#include "recon_tile.h"
#include "zone_ops.h"

namespace ader {

// Ghost zones of bounded problems (non-periodic faces; ader_set_boundary).
// A padded index along an axis of g ghost layers before u interior zones
// maps to the interior zone whose average it takes: outflow the nearest one,
// reflect the mirror image (sign negated for the normal momentum); on an
// inflow face it stays and `inflow` is set to the side (0 lower, 1 upper).
__host__ __device__ __forceinline__ int ghost_source(int i, int g, int u, int lo, int hi,
                                                     double& sign, int& inflow) {
  inflow = -1;
  if (g == 0) return i;
  if (i < g) {
    if (lo == ADER_BC_OUTFLOW) return g;
    if (lo == ADER_BC_INFLOW) {
      inflow = 0;
      return i;
    }
    sign = -sign;
    return 2 * g - 1 - i;
  }
  if (i >= g + u) {
    if (hi == ADER_BC_OUTFLOW) return g + u - 1;
    if (hi == ADER_BC_INFLOW) {
      inflow = 1;
      return i;
    }
    sign = -sign;
    return 2 * (g + u) - 1 - i;
  }
  return i;
}


// A zone two or more layers outside the interior along a bounded axis: its
// polynomials reach no interior face (a step updates only the interior;
// the ghosts are filled again before the next), so its positivity outcome
// goes to the problem's sink slots.
__device__ __forceinline__ bool deep_ghost(const Problem& pr, long long n) {
  if (!(pr.gx | pr.gy | pr.gz)) return false;
  const long long l = n - pr.base;
  const int i = (int)(l % pr.nx), j = (int)((l / pr.nx) % pr.ny);
  const int k = (int)(l / ((long long)pr.nx * pr.ny));
  return (pr.gx && (i < pr.gx - 1 || i > pr.gx + pr.ux)) ||
         (pr.gy && (j < pr.gy - 1 || j > pr.gy + pr.uy)) ||
         (pr.gz && (k < pr.gz - 1 || k > pr.gz + pr.uz));
}

__device__ __forceinline__ PosCtl pos_at(const PosCtl& pc, int p, const Problem& pr, long long n) {
  return deep_ghost(pr, n) ? pc.sunk(p) : pc.at(p);
}

// The FP32 (mixed-precision) kernels run the deviation form, the FP64 ones
// the point form.  Kernels without a natural template parameter take a
// dummy one, so this header can go into several translation units.
template <class T>
constexpr bool kDeviation = sizeof(T) == 4;

__device__ __forceinline__ Grid grid_of(const Problem& pr, const Batch& b) {
  return Grid{pr.nx, pr.ny, pr.nz, pr.N, b.S, pr.base};
}

// Problem holding array index n (the table is sorted by base).
__device__ __forceinline__ int find_problem(const Batch& b, long long n) {
  int lo = 0, hi = b.np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.P[mid].base <= n) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Zone loop of the persistent kernels.  The hardware deals blocks to the 8
// XCDs in turn (block b on XCD b mod 8), so the zone range is cut into 8
// contiguous regions, one per XCD, and each region into contiguous chunks,
// one per block of that XCD: a zone's stencil neighbours (+-1, +-nx, +-nx ny)
// mostly lie in the same region and are read through the same L2.  Threads
// walk their chunk with stride blockDim.x (coalesced) and track the problem
// of the current zone.  Every zone of [0, S) is visited exactly once for any
// grid size.
template <class Body>
__device__ __forceinline__ void for_zones(const Batch& b, Body&& body) {
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long rlo = b.S * x / nreg, rhi = b.S * (x + 1) / nreg;
  const long long lo = rlo + (rhi - rlo) * r / nb, hi = rlo + (rhi - rlo) * (r + 1) / nb;
  long long n = lo + threadIdx.x;
  if (n >= hi) return;
  int p = find_problem(b, n);
  Problem pr = b.P[p];
  for (; n < hi; n += blockDim.x) {
    while (n >= pr.base + pr.N) pr = b.P[++p];
    body(pr, p, n);
  }
}

// Fills the ghost zones of bounded problems from the interior (ghost_source)
// or with the inflow states.  The axes compose in the order x, y, z: a zone
// outside the faces of several axes takes the inflow state of the last of
// them that is an inflow face, with the momentum signs of the reflecting
// axes after it, else the interior source with every axis's sign.
template <int = 0>
__global__ void __launch_bounds__(256) k_fill_ghosts(double* __restrict__ U, Batch b,
                                                     InflowStates in) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    if (!(pr.gx | pr.gy | pr.gz)) return;
    const Grid g = grid_of(pr, b);
    int idx[3];
    zone_ijk(g, n, idx[0], idx[1], idx[2]);
    const int gw[3] = {pr.gx, pr.gy, pr.gz}, uw[3] = {pr.ux, pr.uy, pr.uz};
    double s[3] = {1.0, 1.0, 1.0};
    int src[3], face = -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int side;
      src[d] = ghost_source(idx[d], gw[d], uw[d], pr.bc[2 * d], pr.bc[2 * d + 1], s[d], side);
      if (side >= 0) {
        // the inflow state overrides the axes before this one
        face = 2 * d + side;
#pragma unroll
        for (int e = 0; e <= d; ++e) s[e] = 1.0;
      }
    }
    if (face < 0 && src[0] == idx[0] && src[1] == idx[1] && src[2] == idx[2]) return;   // interior
    double v[5];
    if (face >= 0) {
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = in.v[face][q];
    } else {
      const long long from = zone_of(src[0], src[1], src[2], g);
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = U[(long long)q * b.S + from];
    }
    U[n] = v[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) U[(long long)(1 + d) * b.S + n] = s[d] * v[1 + d];
    U[4 * b.S + n] = v[4];
  });
}

template <class T, int M, int AXIS, int NVAR>
__global__ void __launch_bounds__(256) k_weno_sweep(const double* __restrict__ U,
                                                    T* __restrict__ W, Batch b) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    weno_sweep_zone<T, M, AXIS, NVAR>(U, W, grid_of(pr, b), n);
  });
}

// Tiled reconstruction: tiles in the same XCD-aware order as for_zones (the
// tile range cut into one region per XCD, blocks of an XCD walking theirs),
// so neighbouring tiles, which share halo zones, run on the same L2.
template <class T, int M, int NVAR>
__global__ void __launch_bounds__(256) k_recon_tile(const double* __restrict__ U,
                                                    T* __restrict__ W, Batch b,
                                                    const long long* __restrict__ tile_base) {
  using RT = ReconTile<T, M, NVAR>;
  __shared__ double su[RT::kSu];
  __shared__ T sx[RT::kSx];
  __shared__ T sy[RT::kSy];
  const long long ntiles = tile_base[b.np];
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long lo = ntiles * x / nreg, hi = ntiles * (x + 1) / nreg;
  for (long long t = lo + r; t < hi; t += nb) {
    const int p = problem_of_tile(tile_base, b.np, t);
    const Problem pr = b.P[p];
    const long long lt = t - tile_base[p];
    const int ntx = (pr.nx + kTile - 1) / kTile, nty = (pr.ny + kTile - 1) / kTile;
    const int tx = (int)(lt % ntx), ty = (int)((lt / ntx) % nty);
    const int tz = (int)(lt / ((long long)ntx * nty));
    RT::run(U, W, grid_of(pr, b), tx * kTile, ty * kTile, tz * kTile, su, sx, sy);
  }
}

// z-marching reconstruction: one work item = one variable of kMarchSeg
// planes of one x-y column of kMarchTile^2 zones (items in the XCD-aware
// order of k_recon_tile: the item range cut into one region per XCD)
template <class T, int M, int NVAR>
__global__ void __launch_bounds__(kMarchTile * kMarchTile) k_recon_march(
    const double* __restrict__ U, T* __restrict__ W, Batch b,
    const long long* __restrict__ xy_base) {
  using RM = ReconMarch<T, M, kMarchTile>;
  __shared__ double su[RM::kSu];
  __shared__ T sx[RM::kSx];
  __shared__ double ring0[RM::kRing0];
  __shared__ T ringT[RM::kRingT];
  const long long nitems = xy_base[b.np] * NVAR;
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long lo = nitems * x / nreg, hi = nitems * (x + 1) / nreg;
  for (long long w = lo + r; w < hi; w += nb) {
    const long long q = w / NVAR;
    const int v = (int)(w % NVAR);
    const int p = problem_of_tile(xy_base, b.np, q);
    const Problem pr = b.P[p];
    const Grid g = grid_of(pr, b);
    const long long lt = q - xy_base[p];
    const int ntx = (pr.nx + kMarchTile - 1) / kMarchTile;
    const int nty = (pr.ny + kMarchTile - 1) / kMarchTile;
    const int i0 = (int)(lt % ntx) * kMarchTile, j0 = (int)((lt / ntx) % nty) * kMarchTile;
    const int k0 = (int)(lt / ((long long)ntx * nty)) * kMarchSeg;
    const int k1 = k0 + kMarchSeg < pr.nz ? k0 + kMarchSeg : pr.nz;
    RM::run(U + (long long)v * b.S, W + (long long)v * b.S, g, NVAR, i0, j0, k0, k1, su, sx,
            ring0, ringT);
  }
}

template <class T, int NVAR>
__global__ void __launch_bounds__(256) k_minmod(const double* __restrict__ U, T* __restrict__ W,
                                                Batch b) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    minmod_zone<T, NVAR>(U, W, grid_of(pr, b), n);
  });
}

template <class T, int M>
__global__ void __launch_bounds__(256) k_bface(const double* __restrict__ B, double* __restrict__ B0,
                                               T* __restrict__ BN, Batch b) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    bface_zone<T, M>(B, B0, BN, grid_of(pr, b), n);
  });
}

// a copy of zone n's averages for the fused face-flux+update kernel (the
// deviation-form faces between its blocks read them after the update)
__device__ __forceinline__ void keep_average(const double* __restrict__ U, double* __restrict__ keep,
                                             long long S, long long n) {
#pragma unroll
  for (int v = 0; v < 5; ++v) keep[(long long)v * S + n] = U[(long long)v * S + n];
}

// FUSED: where the facial positivity check runs (see predict_zone); WAVES
// caps the registers for that many waves per SIMD
template <class T, int ORDER, int FORM, bool FUSED, int WAVES = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) k_predict(const double* __restrict__ U,
                                                 const T* __restrict__ W, T* __restrict__ PK,
                                                 Batch b, const double* __restrict__ dt,
                                                 double gam, PosCtl pc,
                                                 double* __restrict__ keep = nullptr) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    if (keep) keep_average(U, keep, b.S, n);
    predict_zone<T, ORDER, FORM, kDeviation<T>, FUSED>(U, W, PK, grid_of(pr, b), dt[p], 1.0 / pr.dx,
                                                       1.0 / pr.dy, 1.0 / pr.dz, gam, pos_at(pc, p, pr, n), n);
  });
}

// Reconstruction and predictor in one kernel (Euler): a block takes tiles of
// kTile x kTile x TZ zones (tiles in the XCD-aware order of k_recon_tile),
// reconstructs each on LDS (ReconLds) and then runs the one-lane-per-zone
// predictor on it, one thread per zone, reading the modes from LDS, so the
// mode array never goes through HBM.  tile_base indexes these tiles.
template <class T, int ORDER, int FORM, int TZ>
__global__ void __launch_bounds__(kTile * kTile * TZ) k_recon_predict(
    const double* __restrict__ U, T* __restrict__ PK, Batch b,
    const long long* __restrict__ tile_base, const double* __restrict__ dt, double gam,
    PosCtl pc, double* __restrict__ keep = nullptr) {
  using RL = ReconLds<T, ORDER, 5, TZ>;
  __shared__ double su[RL::kSu];
  __shared__ T sx[RL::kSx];
  __shared__ T sy[RL::kSy];
  __shared__ T sw[RL::kSw];
  const long long ntiles = tile_base[b.np];
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long lo = ntiles * x / nreg, hi = ntiles * (x + 1) / nreg;
  const int t = threadIdx.x;
  const int tx = t % kTile, ty = (t / kTile) % kTile, tz = t / (kTile * kTile);
  for (long long q = lo + r; q < hi; q += nb) {
    const int p = problem_of_tile(tile_base, b.np, q);
    const Problem pr = b.P[p];
    const Grid g = grid_of(pr, b);
    const long long lt = q - tile_base[p];
    const int ntx = (pr.nx + kTile - 1) / kTile, nty = (pr.ny + kTile - 1) / kTile;
    const int i0 = (int)(lt % ntx) * kTile, j0 = (int)((lt / ntx) % nty) * kTile;
    const int k0 = (int)(lt / ((long long)ntx * nty)) * TZ;
    RL::run(U, g, i0, j0, k0, su, sx, sy, sw);
    if (i0 + tx < pr.nx && j0 + ty < pr.ny && k0 + tz < pr.nz) {
      const long long n = zone_of(i0 + tx, j0 + ty, k0 + tz, g);
      if (keep) keep_average(U, keep, g.S, n);
      predict_zone_lds<T, ORDER, FORM, kDeviation<T>>(U, sw + t, RL::NZ, PK, g, dt[p],
                                                      1.0 / pr.dx, 1.0 / pr.dy, 1.0 / pr.dz, gam,
                                                      pos_at(pc, p, pr, n), n);
    }
    __syncthreads();   // the next tile overwrites the LDS
  }
}

// linear advection (test system): predictor and face fluxes
template <class T, int ORDER, int FORM>
__global__ void __launch_bounds__(256) k_predict_adv(const double* __restrict__ U,
                                                     const T* __restrict__ W, T* __restrict__ PK,
                                                     Batch b, const double* __restrict__ dt,
                                                     double ax, double ay, double az) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    predict_zone_adv<T, ORDER, FORM>(U, W, PK, grid_of(pr, b), dt[p], 1.0 / pr.dx, 1.0 / pr.dy,
                                     1.0 / pr.dz, ax, ay, az, n);
  });
}

template <class T>
__global__ void __launch_bounds__(256) k_face_flux_adv(const T* __restrict__ PK,
                                                       double* __restrict__ F, Batch b, double ax,
                                                       double ay, double az) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    face_flux_adv_zone<T>(PK, F, grid_of(pr, b), ax, ay, az, n);
  });
}

// the one-lane-per-zone predictor with the affine source term; dt S-bar to SB
template <class T, int ORDER, int FORM>
__global__ void __launch_bounds__(256) k_predict_src(const double* __restrict__ U,
                                                     const T* __restrict__ W, T* __restrict__ PK,
                                                     Batch b, const double* __restrict__ dt,
                                                     double gam, PosCtl pc, SourceAffine src,
                                                     double* __restrict__ SB) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    predict_zone<T, ORDER, FORM, kDeviation<T>, true, true>(U, W, PK, grid_of(pr, b), dt[p],
                                                            1.0 / pr.dx, 1.0 / pr.dy, 1.0 / pr.dz,
                                                            gam, pos_at(pc, p, pr, n), n, &src, SB);
  });
}

// EDGES_ALL: the side packets carry every variable's edge averages
template <class T, int ORDER, int FORM, bool FUSED, bool EDGES_ALL>
__global__ void __launch_bounds__(256) k_predict_mhd(const double* __restrict__ U,
                                                     const T* __restrict__ W,
                                                     const double* __restrict__ B0,
                                                     const T* __restrict__ WB,
                                                     const T* __restrict__ BN, T* __restrict__ PK,
                                                     Batch b, const double* __restrict__ dt,
                                                     double gam, PosCtl pc) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    predict_zone_mhd<T, ORDER, FORM, kDeviation<T>, FUSED, EDGES_ALL>(U, W, B0, WB, BN, PK, grid_of(pr, b),
                                                           dt[p], 1.0 / pr.dx, 1.0 / pr.dy,
                                                           1.0 / pr.dz, gam, pos_at(pc, p, pr, n), n);
  });
}

// Zone loop of the lane-split kernels: the same chunks as for_zones, walked
// Z = 64 / NV zones per wave and step, lane var * Z + z on zone slot z.
// Lanes past NV Z (when 64 is not a multiple of NV) stay idle.
template <int NV, class Body>
__device__ __forceinline__ void for_zone_groups(const Batch& b, Body&& body) {
  constexpr int Z = 64 / NV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const SplitLane L{lane / Z, lane % Z, Z};
  if (L.var >= NV) return;
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long rlo = b.S * x / nreg, rhi = b.S * (x + 1) / nreg;
  const long long lo = rlo + (rhi - rlo) * r / nb, hi = rlo + (rhi - rlo) * (r + 1) / nb;
  long long n = lo + (long long)wave * Z + L.z;
  if (n >= hi) return;
  int p = find_problem(b, n);
  Problem pr = b.P[p];
  for (; n < hi; n += (long long)nw * Z) {
    while (n >= pr.base + pr.N) pr = b.P[++p];
    body(L, pr, p, n);
  }
}

// WAVES: the compiler keeps the registers low enough for that many waves
// per SIMD (1: no cap); the autotuner picks between the instances.
template <class T, int ORDER, int FORM, int WAVES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) k_predict_split(const double* __restrict__ U,
                                                       const T* __restrict__ W, T* __restrict__ PK,
                                                       Batch b, const double* __restrict__ dt,
                                                       double gam, PosCtl pc,
                                                       double* __restrict__ keep = nullptr) {
  for_zone_groups<5>(b, [&](const SplitLane& L, const Problem& pr, int p, long long n) {
    if (keep) keep[(long long)L.var * b.S + n] = U[(long long)L.var * b.S + n];
    predict_zone_split<T, ORDER, FORM, kDeviation<T>>(L, U, W, PK, grid_of(pr, b), dt[p],
                                                      1.0 / pr.dx, 1.0 / pr.dy, 1.0 / pr.dz, gam,
                                                      pos_at(pc, p, pr, n), n);
  });
}

// the lane-split predictor with the affine source term; dt S-bar to SB
template <class T, int ORDER, int FORM>
__global__ void __launch_bounds__(256) k_predict_split_src(const double* __restrict__ U,
                                                           const T* __restrict__ W,
                                                           T* __restrict__ PK, Batch b,
                                                           const double* __restrict__ dt,
                                                           double gam, PosCtl pc,
                                                           SourceAffine src,
                                                           double* __restrict__ SB) {
  for_zone_groups<5>(b, [&](const SplitLane& L, const Problem& pr, int p, long long n) {
    predict_zone_split<T, ORDER, FORM, kDeviation<T>, true>(L, U, W, PK, grid_of(pr, b), dt[p],
                                                            1.0 / pr.dx, 1.0 / pr.dy,
                                                            1.0 / pr.dz, gam, pos_at(pc, p, pr, n), n, &src,
                                                            SB);
  });
}

template <class T, int ORDER, int FORM, int WAVES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) k_predict_mhd_split(
    const double* __restrict__ U, const T* __restrict__ W, const double* __restrict__ B0,
    const T* __restrict__ WB, const T* __restrict__ BN, T* __restrict__ PK, Batch b,
    const double* __restrict__ dt, double gam, PosCtl pc) {
  for_zone_groups<8>(b, [&](const SplitLane& L, const Problem& pr, int p, long long n) {
    predict_zone_mhd_split<T, ORDER, FORM, kDeviation<T>>(L, U, W, B0, WB, BN, PK, grid_of(pr, b),
                                                          dt[p], 1.0 / pr.dx, 1.0 / pr.dy,
                                                          1.0 / pr.dz, gam, pos_at(pc, p, pr, n), n);
  });
}

// z sweep by column segments: thread t -> problem p (seg_base), then i
// fastest, j, segment; one segment of kZSeg planes per thread
template <class T, int M, int NVAR>
__global__ void __launch_bounds__(256) k_weno_z_columns(const double* __restrict__ U,
                                                        T* __restrict__ W, Batch b,
                                                        const long long* __restrict__ seg_base) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= seg_base[b.np]) return;
  const int p = problem_of_tile(seg_base, b.np, t);
  const Problem pr = b.P[p];
  const long long local = t - seg_base[p];
  const int i = (int)(local % pr.nx);
  const long long r = local / pr.nx;
  const int j = (int)(r % pr.ny);
  const int s = (int)(r / pr.ny);
  const int k0 = s * kZSeg;
  const int k1 = k0 + kZSeg < pr.nz ? k0 + kZSeg : pr.nz;
  ZColumn<T, M, NVAR>::run(U, W, grid_of(pr, b), i, j, k0, k1);
}

// SSP-RK stage (Euler): side packets of the spatial polynomial
template <class T, int ORDER>
__global__ void __launch_bounds__(256) k_rk_sides(const double* __restrict__ U,
                                                  const T* __restrict__ W, T* __restrict__ PK,
                                                  Batch b, double gam, PosCtl pc) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    rk_sides_zone<T, ORDER, kDeviation<T>>(U, W, PK, grid_of(pr, b), gam, pos_at(pc, p, pr, n), n);
  });
}

// SSP-RK stage combination (eq. 18-20)
template <int = 0>
__global__ void __launch_bounds__(256) k_rk_stage(double* __restrict__ U,
                                                  const double* __restrict__ F, RkStage st,
                                                  Batch b, const double* __restrict__ dt) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    rk_stage_zone(U, F, st, grid_of(pr, b), dt[p], pr.dx, pr.dy, pr.dz, n);
  });
}

// SSP-RK stage (MHD): side packets of the spatial polynomial
template <class T, int ORDER, bool EDGES_ALL>
__global__ void __launch_bounds__(256) k_rk_sides_mhd(const double* __restrict__ U,
                                                      const T* __restrict__ W,
                                                      const double* __restrict__ B0,
                                                      const T* __restrict__ WB,
                                                      const T* __restrict__ BN,
                                                      T* __restrict__ PK, Batch b, double gam,
                                                      PosCtl pc) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    predict_zone_mhd<T, ORDER, 0, kDeviation<T>, true, EDGES_ALL, true>(
        U, W, B0, WB, BN, PK, grid_of(pr, b), 0.0, 0.0, 0.0, 0.0, gam, pos_at(pc, p, pr, n), n);
  });
}

// SSP-RK stage combination of the MHD face fields
template <int = 0>
__global__ void __launch_bounds__(256) k_rk_stage_field(double* __restrict__ B,
                                                        const double* __restrict__ E, RkStage st,
                                                        Batch b, const double* __restrict__ dt) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    rk_stage_field_zone(B, E, st, grid_of(pr, b), dt[p], pr.dx, pr.dy, pr.dz, n);
  });
}

// dst <- src for `rows` state rows (the step's starting state of SSP-RK)
template <int = 0>
__global__ void __launch_bounds__(256) k_copy_state(const double* __restrict__ src,
                                                    double* __restrict__ dst, int rows, Batch b) {
  for_zones(b, [&](const Problem&, int, long long n) {
    for (int v = 0; v < rows; ++v) dst[(long long)v * b.S + n] = src[(long long)v * b.S + n];
  });
}

// pair layout (MHD): two lanes per zone, 32 zones per wave; PHASE as in
// predict_zone_mhd_pair (0: whole, 1: predictor, 2: side packets)
template <class T, int ORDER, int FORM, int WAVES, bool EDGES_ALL, int PHASE = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) k_predict_mhd_pair(
    const double* __restrict__ U, const T* __restrict__ W, const double* __restrict__ B0,
    const T* __restrict__ WB, const T* __restrict__ BN, T* __restrict__ PK, Batch b,
    const double* __restrict__ dt, double gam, PosCtl pc, T* __restrict__ EM = nullptr,
    double* __restrict__ TH = nullptr) {
  for_zone_groups<2>(b, [&](const SplitLane& L, const Problem& pr, int p, long long n) {
    predict_zone_mhd_pair<T, ORDER, FORM, kDeviation<T>, EDGES_ALL, PHASE>(
        L, U, W, B0, WB, BN, PK, grid_of(pr, b), dt[p], 1.0 / pr.dx, 1.0 / pr.dy, 1.0 / pr.dz,
        gam, pos_at(pc, p, pr, n), n, EM, TH);
  });
}

template <class T, int RS>
__global__ void __launch_bounds__(256) k_face_flux(const double* __restrict__ U,
                                                   const T* __restrict__ PK,
                                                   double* __restrict__ F, Batch b, double gam) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    face_flux_zone<T, RS, kDeviation<T>>(U, PK, F, grid_of(pr, b), gam, n);
  });
}

// Face fluxes and the update of eq. (6) in one kernel (Euler).  A work item
// is an x-y tile of kFuTX x kFuTY zones and a segment of kFuSeg planes; the
// block walks it in z.  Per plane each thread forms its zone's lower x and y
// faces into LDS and its upper z face into registers (the lower z face is
// the previous plane's upper one; the segment's first lower z face and the
// tile's upper x and y faces are formed here too, and again by the block
// that owns their other zone), then updates its zone from them.  Every face
// is formed by face_flux_values, as in k_face_flux, and the update takes
// update_zone's order of operations, so the two paths agree bit for bit,
// while no flux reaches device memory.  With deviation-form packets a face
// needs the zone averages at the step's start, also of zones that another
// block updates meanwhile: those come from the copy U0 the predictor keeps
// (read for the block's own zones too, so a launch can be repeated).
template <class T, int RS>
__global__ void __launch_bounds__(kFuTX * kFuTY) k_flux_update(
    double* __restrict__ U, const double* __restrict__ U0, const T* __restrict__ PK, Batch b,
    const long long* __restrict__ fu_base, const double* __restrict__ dt, double gam) {
  constexpr bool DEV = kDeviation<T>;
  static_assert(kFuTY <= 64 && kFuTX <= 64 && kFuTX * kFuTY >= 64 + kFuTX,
                "the tile's upper faces are formed by waves 0 and 1");
  __shared__ double fx[5][kFuTY][kFuTX + 1];   // x faces: [v][row j][lower face of local zone i]
  __shared__ double fy[5][kFuTY + 1][kFuTX];   // y faces: [v][lower face of local row j][i]
  const double* UA = DEV ? U0 : U;             // the averages the faces and the update read
  const long long nitems = fu_base[b.np];
  const int G = gridDim.x;
  const int nreg = G < 8 ? G : 8;
  const int x = blockIdx.x % nreg, r = blockIdx.x / nreg;
  const int nb = (G - x + nreg - 1) / nreg;
  const long long lo = nitems * x / nreg, hi = nitems * (x + 1) / nreg;
  const int t = threadIdx.x, ti = t % kFuTX, tj = t / kFuTX;
  for (long long q = lo + r; q < hi; q += nb) {
    const int p = problem_of_tile(fu_base, b.np, q);
    const Problem pr = b.P[p];
    const Grid g = grid_of(pr, b);
    const long long lt = q - fu_base[p];
    const int ntx = (pr.nx + kFuTX - 1) / kFuTX, nty = (pr.ny + kFuTY - 1) / kFuTY;
    const int i0 = (int)(lt % ntx) * kFuTX, j0 = (int)((lt / ntx) % nty) * kFuTY;
    const int k0 = (int)(lt / ((long long)ntx * nty)) * kFuSeg;
    const int k1 = k0 + kFuSeg < pr.nz ? k0 + kFuSeg : pr.nz;
    const int i = i0 + ti, j = j0 + tj;
    const bool in = i < pr.nx && j < pr.ny;
    // local index of the tile's upper x face (y face): the upper face of its
    // last zone, shared with the next zone (periodically wrapped)
    const int ex = pr.nx - i0 < kFuTX ? pr.nx - i0 : kFuTX;
    const int ey = pr.ny - j0 < kFuTY ? pr.ny - j0 : kFuTY;
    const double h = dt[p];
    const double c[3] = {h / pr.dx, h / pr.dy, h / pr.dz};
    double fzl[5], fzu[5], res[5];
    if (in)
      face_flux_values<T, RS, 2, DEV>(UA, PK, g, zone_of(i, j, k0, g),
                                      zone_of(i, j, wrap(k0 - 1, g.nz), g), gam, fzl);
    for (int k = k0; k < k1; ++k) {
      if (in) {
        const long long n = zone_of(i, j, k, g);
        face_flux_values<T, RS, 0, DEV>(UA, PK, g, n, zone_of(wrap(i - 1, g.nx), j, k, g), gam, res);
#pragma unroll
        for (int v = 0; v < 5; ++v) fx[v][tj][ti] = res[v];
        face_flux_values<T, RS, 1, DEV>(UA, PK, g, n, zone_of(i, wrap(j - 1, g.ny), k, g), gam, res);
#pragma unroll
        for (int v = 0; v < 5; ++v) fy[v][tj][ti] = res[v];
        face_flux_values<T, RS, 2, DEV>(UA, PK, g, zone_of(i, j, wrap(k + 1, g.nz), g), n, gam, fzu);
      }
      if (t < ey) {
        // wave 0: the upper x face of row t
        face_flux_values<T, RS, 0, DEV>(UA, PK, g, zone_of(wrap(i0 + ex, g.nx), j0 + t, k, g),
                                        zone_of(i0 + ex - 1, j0 + t, k, g), gam, res);
#pragma unroll
        for (int v = 0; v < 5; ++v) fx[v][t][ex] = res[v];
      } else if (t >= 64 && t < 64 + ex) {
        // wave 1: the upper y face of column t - 64
        const int il = t - 64;
        face_flux_values<T, RS, 1, DEV>(UA, PK, g, zone_of(i0 + il, wrap(j0 + ey, g.ny), k, g),
                                        zone_of(i0 + il, j0 + ey - 1, k, g), gam, res);
#pragma unroll
        for (int v = 0; v < 5; ++v) fy[v][ey][il] = res[v];
      }
      __syncthreads();
      if (in) {
#pragma clang fp contract(on)   // as update_zone: equal bits
        // eq. (6) in update_zone's order: per variable x, then y, then z
        const long long n = zone_of(i, j, k, g);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          double u = UA[(long long)v * g.S + n];
          u = u - c[0] * (fx[v][tj][ti + 1] - fx[v][tj][ti]);
          u = u - c[1] * (fy[v][tj + 1][ti] - fy[v][tj][ti]);
          u = u - c[2] * (fzu[v] - fzl[v]);
          U[(long long)v * g.S + n] = u;
          fzl[v] = fzu[v];
        }
      }
      __syncthreads();   // the next plane overwrites the LDS faces
    }
  }
}

template <class T, int RS>
__global__ void __launch_bounds__(256) k_face_flux_mhd(const double* __restrict__ U,
                                                       const double* __restrict__ B0,
                                                       const T* __restrict__ PK,
                                                       double* __restrict__ F,
                                                       double* __restrict__ FE, Batch b,
                                                       double gam) {
  for_zones(b, [&](const Problem& pr, int, long long n) {
    face_flux_zone_mhd<T, RS, kDeviation<T>>(U, B0, PK, F, FE, grid_of(pr, b), gam, n);
  });
}

template <int = 0>
__global__ void __launch_bounds__(256) k_edge_e(const double* __restrict__ FE,
                                                double* __restrict__ E, Batch b) {
  for_zones(b, [&](const Problem& pr, int, long long n) { edge_e_zone(FE, E, grid_of(pr, b), n); });
}

// eq. (6)
template <int = 0>
__global__ void __launch_bounds__(256) k_update(double* __restrict__ U, const double* __restrict__ F,
                                                Batch b, const double* __restrict__ dt) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    update_zone(U, F, grid_of(pr, b), dt[p], pr.dx, pr.dy, pr.dz, n);
  });
}

// eq. (6) with the source term dt S-bar
template <int = 0>
__global__ void __launch_bounds__(256) k_update_src(double* __restrict__ U,
                                                    const double* __restrict__ F,
                                                    const double* __restrict__ SB, Batch b,
                                                    const double* __restrict__ dt) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    const Grid g = grid_of(pr, b);
    update_zone(U, F, g, dt[p], pr.dx, pr.dy, pr.dz, n);
    source_zone(U, SB, g, n);
  });
}

// eq. (6) for the hydro variables and eq. (8) for the face fields
template <int = 0>
__global__ void __launch_bounds__(256) k_update_mhd(double* __restrict__ U, double* __restrict__ B,
                                                    const double* __restrict__ F,
                                                    const double* __restrict__ E, Batch b,
                                                    const double* __restrict__ dt) {
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    const Grid g = grid_of(pr, b);
    update_zone(U, F, g, dt[p], pr.dx, pr.dy, pr.dz, n);
    ct_zone(B, E, g, dt[p], pr.dx, pr.dy, pr.dz, n);
  });
}

// ---------------------------------------------------------------------------
// CFL dt per problem: every zone's rate sum_d (|v_d| + c_d)/dx_d is maxed into
// rate[p] (the bit pattern of a non-negative double orders like the value,
// so an unsigned 64-bit atomic max is a max of doubles).  A block's threads
// keep a running max for their current problem and flush it when the
// problem changes; at the end the wave and then the block combine the
// maxima of equal problems, so a block issues one atomic per problem it
// touched.  k_dt_final turns the rates into dt and clears them for the next
// step (no memset, so the step can be captured in a graph).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void flush_rate(unsigned long long* rate, int p, double r) {
  if (p >= 0 && r > 0.0) atomicMax(&rate[p], (unsigned long long)__double_as_longlong(r));
}

template <int = 0>
__global__ void __launch_bounds__(256) k_dt(const double* __restrict__ U,
                                            const double* __restrict__ B, Batch b, double gam,
                                            unsigned long long* __restrict__ rate,
                                            int* __restrict__ bad) {
  __shared__ int sp[4];
  __shared__ double sr[4];
  double rmax = 0.0;
  int pcur = -1;
  for_zones(b, [&](const Problem& pr, int p, long long n) {
    if (p != pcur) {
      flush_rate(rate, pcur, rmax);
      rmax = 0.0;
      pcur = p;
    }
    int isbad = 0;
    const Grid g = grid_of(pr, b);
    const double r = B ? dt_rate_zone_mhd(U, B, g, gam, pr.dx, pr.dy, pr.dz, n, isbad)
                       : dt_rate_zone(U, g, gam, pr.dx, pr.dy, pr.dz, n, isbad);
    if (isbad) bad[p] = 1;
    rmax = fmax(rmax, r);
  });
  // wave: lanes that agree on the problem (idle lanes hold -1) combine
  int pmax = pcur, pmin = pcur < 0 ? 0x7fffffff : pcur;
  for (int off = 32; off >= 1; off >>= 1) {
    pmax = max(pmax, __shfl_xor(pmax, off, 64));
    pmin = min(pmin, __shfl_xor(pmin, off, 64));
  }
  const bool uniform = pmax >= 0 && pmin == pmax;
  double rw = uniform ? rmax : 0.0;
  for (int off = 32; off >= 1; off >>= 1) rw = fmax(rw, __shfl_xor(rw, off, 64));
  if (!uniform) flush_rate(rate, pcur, rmax);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sp[wid] = uniform ? pmax : -1;
    sr[wid] = rw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    int p = -1;
    double r = 0.0;
    for (int q = 0; q < nw; ++q) {
      if (sp[q] != p) {
        flush_rate(rate, p, r);
        p = sp[q];
        r = 0.0;
      }
      r = fmax(r, sr[q]);
    }
    flush_rate(rate, p, r);
  }
}

template <int = 0>
__global__ void __launch_bounds__(64) k_dt_final(unsigned long long* __restrict__ rate,
                                                 int* __restrict__ bad, int np, double cfl,
                                                 double* __restrict__ dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double r = __longlong_as_double((long long)rate[p]);
  if (!(r > 0.0) || !__builtin_isfinite(r)) bad[p] = 1;
  else if (!bad[p]) dt[p] = cfl / r;
  rate[p] = 0ull;
}

// dt of linear advection per problem: cfl / sum_d |a_d| / dx_d
template <int = 0>
__global__ void __launch_bounds__(64) k_dt_adv(Batch b, double cfl, double ax, double ay,
                                               double az, double* __restrict__ dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.np) return;
  const Problem pr = b.P[p];
  dt[p] = cfl / (fabs(ax) / pr.dx + fabs(ay) / pr.dy + fabs(az) / pr.dz);
}

template <int = 0>
__global__ void __launch_bounds__(64) k_set_dt(double* __restrict__ dt, int np, double value) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) dt[p] = value;
}

}  // namespace ader
