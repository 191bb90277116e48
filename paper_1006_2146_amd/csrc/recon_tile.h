// Reconstruction on LDS tiles (device only): the x, y and z sweeps of the
// centred WENO reconstruction (Sec. II.1; the reading of all M-zone
// stencils, x -> y -> z) for a tile of 8 x 8 x 8 zones in one kernel.  The
// zone averages of the tile and its halo of M-1 zones are staged in LDS; the
// x sweep runs on the tile widened by the halo in y and z, the y sweep on
// the tile widened in z, the z sweep on the tile, each reading the previous
// sweep's moments from LDS, and every moment is written to HBM once.  Each
// line is reconstructed by the same weno1d on the same inputs as in the
// one-sweep-per-kernel path; the compiler may contract its multiply-adds
// differently in the two kernels, so the modes agree to rounding.
#pragma once
#include <hip/hip_runtime.h>

#include "zone_ops.h"

namespace ader {

constexpr int kTile = 8;   // zones per tile edge
constexpr int kFusedTZ = 4;   // z depth of the fused reconstruction+predictor's tiles
constexpr int kMarchTile = 16;   // x-y edge of the z-marching reconstruction's columns
constexpr int kMarchSeg = 32;    // z planes per work item of that reconstruction

// (a, b) with b >= 1 and a + b <= M - 1, in the order a, then b
template <int M>
__host__ __device__ constexpr int ymoment_slot(int a, int b) {
  int s = 0;
  for (int aa = 0; aa <= M - 2; ++aa)
    for (int bb = 1; aa + bb <= M - 1; ++bb) {
      if (aa == a && bb == b) return s;
      ++s;
    }
  return -1;
}

// Tiles of problem p: tile_base[p] .. tile_base[p+1]-1; tile t -> (p, tx, ty, tz)
__device__ __forceinline__ int problem_of_tile(const long long* __restrict__ tile_base, int np,
                                               long long t) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_base[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T, int M, int NVAR>
struct ReconTile {
  static constexpr int R = M - 1;
  static constexpr int EX = kTile + 2 * R, EY = kTile + 2 * R, EZ = kTile + 2 * R;
  static constexpr int NXF = M - 1;             // x-moment fields a = 1..M-1
  static constexpr int NYF = M * (M - 1) / 2;   // y-moment fields (a, b), b >= 1
  static constexpr int kSu = EZ * EY * EX;
  static constexpr int kSx = NXF * EZ * EY * kTile;
  static constexpr int kSy = NYF * EZ * kTile * kTile;

  // One tile: origin (i0, j0, k0) of problem g; su, sx, sy in LDS.
  __device__ static void run(const double* __restrict__ U, T* __restrict__ W, const Grid& g,
                             int i0, int j0, int k0, double* su, T* sx, T* sy) {
    for (int v = 0; v < NVAR; ++v) {
      const double* Uv = U + (long long)v * g.S;
      for (int e = threadIdx.x; e < kSu; e += blockDim.x) {
        const int x = e % EX, y = (e / EX) % EY, z = e / (EX * EY);
        su[e] = Uv[zone_of(wrap(i0 + x - R, g.nx), wrap(j0 + y - R, g.ny), wrap(k0 + z - R, g.nz), g)];
      }
      __syncthreads();
      // x sweep on kTile x EY x EZ: moments (a, 0, 0)
      for (int e = threadIdx.x; e < kTile * EY * EZ; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % EY, z = e / (kTile * EY);
        const double* row = su + (z * EY + y) * EX + x;
        const double c = row[R];
        T d[2 * M - 1];
#pragma unroll
        for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(row[q] - c);
        T m[M];
        weno1d<T, M>(d, m);
        const bool inside = y >= R && y < R + kTile && z >= R && z < R + kTile &&
                            i0 + x < g.nx && j0 + y - R < g.ny && k0 + z - R < g.nz;
        const long long n = inside ? zone_of(i0 + x, j0 + y - R, k0 + z - R, g) : 0;
#pragma unroll
        for (int a = 1; a <= M - 1; ++a) {
          sx[(((a - 1) * EZ + z) * EY + y) * kTile + x] = m[a];
          if (inside) W[((long long)(spatial_mode(a, 0, 0) - 1) * NVAR + v) * g.S + n] = m[a];
        }
      }
      __syncthreads();
      // y sweep on kTile x kTile x EZ of the fields (a, 0), a <= M-2: (a, b, 0)
      for (int e = threadIdx.x; e < kTile * kTile * EZ; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % kTile, z = e / (kTile * kTile);
        const bool inside = z >= R && z < R + kTile && i0 + x < g.nx && j0 + y < g.ny &&
                            k0 + z - R < g.nz;
        const long long n = inside ? zone_of(i0 + x, j0 + y, k0 + z - R, g) : 0;
#pragma unroll
        for (int a = 0; a <= M - 2; ++a) {
          T d[2 * M - 1];
          if (a == 0) {
            const double c = su[(z * EY + y + R) * EX + x + R];
#pragma unroll
            for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(su[(z * EY + y + q) * EX + x + R] - c);
          } else {
#pragma unroll
            for (int q = 0; q < 2 * M - 1; ++q) d[q] = sx[(((a - 1) * EZ + z) * EY + y + q) * kTile + x];
          }
          T m[M];
          weno1d<T, M>(d, m);
#pragma unroll
          for (int bb = 1; bb <= M - 1 - a; ++bb) {
            sy[((ymoment_slot<M>(a, bb) * EZ + z) * kTile + y) * kTile + x] = m[bb];
            if (inside) W[((long long)(spatial_mode(a, bb, 0) - 1) * NVAR + v) * g.S + n] = m[bb];
          }
        }
      }
      __syncthreads();
      // z sweep on the tile of the fields (a, b, 0), a + b <= M-2: (a, b, c)
      for (int e = threadIdx.x; e < kTile * kTile * kTile; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % kTile, z = e / (kTile * kTile);
        const bool inside = i0 + x < g.nx && j0 + y < g.ny && k0 + z < g.nz;
        if (!inside) continue;
        const long long n = zone_of(i0 + x, j0 + y, k0 + z, g);
#pragma unroll
        for (int a = 0; a <= M - 2; ++a)
#pragma unroll
          for (int bb = 0; a + bb <= M - 2; ++bb) {
            T d[2 * M - 1];
            if (a == 0 && bb == 0) {
              const double c = su[((z + R) * EY + y + R) * EX + x + R];
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(su[((z + q) * EY + y + R) * EX + x + R] - c);
            } else if (bb == 0) {
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q)
                d[q] = sx[(((a - 1) * EZ + z + q) * EY + y + R) * kTile + x];
            } else {
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q)
                d[q] = sy[((ymoment_slot<M>(a, bb) * EZ + z + q) * kTile + y) * kTile + x];
            }
            T m[M];
            weno1d<T, M>(d, m);
#pragma unroll
            for (int cc = 1; cc <= M - 1 - a - bb; ++cc)
              W[((long long)(spatial_mode(a, bb, cc) - 1) * NVAR + v) * g.S + n] = m[cc];
          }
      }
      __syncthreads();
    }
  }
};

// The same three sweeps on a tile of kTile x kTile x TZ zones whose modes
// stay in LDS for a predictor in the same kernel: mode m (1..L_S-1) of
// variable v of tile zone t = (z kTile + y) kTile + x at
// sw[((m - 1) NVAR + v) NZ + t], NZ = kTile^2 TZ.  Halo zones come from the
// periodic wrap; zones of a partial tile past the problem's edge get
// reconstructions of wrapped data that nothing reads.
template <class T, int M, int NVAR, int TZ>
struct ReconLds {
  static constexpr int R = M - 1;
  static constexpr int EX = kTile + 2 * R, EY = kTile + 2 * R, EZ = TZ + 2 * R;
  static constexpr int NXF = M - 1;
  static constexpr int NYF = M * (M - 1) / 2;
  static constexpr int NZ = kTile * kTile * TZ;
  static constexpr int LS = M * (M + 1) * (M + 2) / 6;
  static constexpr int kSu = EZ * EY * EX;
  static constexpr int kSx = NXF * EZ * EY * kTile;
  static constexpr int kSy = NYF * EZ * kTile * kTile;
  static constexpr int kSw = (LS - 1) * NVAR * NZ;

  __device__ static void run(const double* __restrict__ U, const Grid& g, int i0, int j0, int k0,
                             double* su, T* sx, T* sy, T* sw) {
    for (int v = 0; v < NVAR; ++v) {
      const double* Uv = U + (long long)v * g.S;
      for (int e = threadIdx.x; e < kSu; e += blockDim.x) {
        const int x = e % EX, y = (e / EX) % EY, z = e / (EX * EY);
        su[e] = Uv[zone_of(wrap(i0 + x - R, g.nx), wrap(j0 + y - R, g.ny), wrap(k0 + z - R, g.nz), g)];
      }
      __syncthreads();
      // x sweep on kTile x EY x EZ: moments (a, 0, 0)
      for (int e = threadIdx.x; e < kTile * EY * EZ; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % EY, z = e / (kTile * EY);
        const double* row = su + (z * EY + y) * EX + x;
        const double c = row[R];
        T d[2 * M - 1];
#pragma unroll
        for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(row[q] - c);
        T m[M];
        weno1d<T, M>(d, m);
        const bool inside = y >= R && y < R + kTile && z >= R && z < R + TZ;
        const int t = ((z - R) * kTile + (y - R)) * kTile + x;
#pragma unroll
        for (int a = 1; a <= M - 1; ++a) {
          sx[(((a - 1) * EZ + z) * EY + y) * kTile + x] = m[a];
          if (inside) sw[((spatial_mode(a, 0, 0) - 1) * NVAR + v) * NZ + t] = m[a];
        }
      }
      __syncthreads();
      // y sweep on kTile x kTile x EZ of the fields (a, 0), a <= M-2: (a, b, 0)
      for (int e = threadIdx.x; e < kTile * kTile * EZ; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % kTile, z = e / (kTile * kTile);
        const bool inside = z >= R && z < R + TZ;
        const int t = ((z - R) * kTile + y) * kTile + x;
#pragma unroll
        for (int a = 0; a <= M - 2; ++a) {
          T d[2 * M - 1];
          if (a == 0) {
            const double c = su[(z * EY + y + R) * EX + x + R];
#pragma unroll
            for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(su[(z * EY + y + q) * EX + x + R] - c);
          } else {
#pragma unroll
            for (int q = 0; q < 2 * M - 1; ++q) d[q] = sx[(((a - 1) * EZ + z) * EY + y + q) * kTile + x];
          }
          T m[M];
          weno1d<T, M>(d, m);
#pragma unroll
          for (int bb = 1; bb <= M - 1 - a; ++bb) {
            sy[((ymoment_slot<M>(a, bb) * EZ + z) * kTile + y) * kTile + x] = m[bb];
            if (inside) sw[((spatial_mode(a, bb, 0) - 1) * NVAR + v) * NZ + t] = m[bb];
          }
        }
      }
      __syncthreads();
      // z sweep on the tile of the fields (a, b, 0), a + b <= M-2: (a, b, c)
      for (int e = threadIdx.x; e < NZ; e += blockDim.x) {
        const int x = e % kTile, y = (e / kTile) % kTile, z = e / (kTile * kTile);
#pragma unroll
        for (int a = 0; a <= M - 2; ++a)
#pragma unroll
          for (int bb = 0; a + bb <= M - 2; ++bb) {
            T d[2 * M - 1];
            if (a == 0 && bb == 0) {
              const double c = su[((z + R) * EY + y + R) * EX + x + R];
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(su[((z + q) * EY + y + R) * EX + x + R] - c);
            } else if (bb == 0) {
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q)
                d[q] = sx[(((a - 1) * EZ + z + q) * EY + y + R) * kTile + x];
            } else {
#pragma unroll
              for (int q = 0; q < 2 * M - 1; ++q)
                d[q] = sy[((ymoment_slot<M>(a, bb) * EZ + z + q) * kTile + y) * kTile + x];
            }
            T m[M];
            weno1d<T, M>(d, m);
#pragma unroll
            for (int cc = 1; cc <= M - 1 - a - bb; ++cc)
              sw[((spatial_mode(a, bb, cc) - 1) * NVAR + v) * NZ + e] = m[cc];
          }
      }
      __syncthreads();
    }
  }
};

// One-pass reconstruction marching in z: a block takes one variable of an
// x-y tile of TXY x TXY zones and walks the whole z column plane by plane.
// For each new plane p it stages the plane's zone averages with an x-y halo
// of R = M-1 zones in LDS, runs the x and y sweeps in the plane (writing the
// modes (a,0,0) and (a,b,0)) and keeps the z-sweep sources of the plane,
// (a,b,0) with a+b <= M-2, in a ring of 2R+1 planes; the z sweep of plane
// p-R then reads its window from the ring and writes the modes (a,b,c),
// c >= 1.  The zone averages are read about once ((TXY+2R)^2 / TXY^2 per
// plane) and every mode is written once.  Each line is reconstructed by the
// same weno1d on the same inputs as in the one-sweep-per-kernel path.
template <class T, int M, int TXY>
struct ReconMarch {
  static constexpr int R = M - 1, NW = 2 * R + 1;
  static constexpr int E = TXY + 2 * R;               // staged plane edge
  static constexpr int NXS = M - 2;                   // x fields (a,0) feeding the y sweep
  static constexpr int NSRC = M * (M - 1) / 2;        // z sources (a,b), incl. (0,0)
  static constexpr int kSu = E * E;
  static constexpr int kSx = (NXS > 0 ? NXS : 1) * E * TXY;
  static constexpr int kRing0 = NW * TXY * TXY;       // (0,0): zone averages, double
  static constexpr int kRingT = NW * (NSRC - 1) * TXY * TXY;

  __host__ __device__ static constexpr int src_a(int s) {
    int q = 0;
    for (int a = 0; a <= M - 2; ++a)
      for (int b = 0; a + b <= M - 2; ++b) {
        if (q == s) return a;
        ++q;
      }
    return -1;
  }
  __host__ __device__ static constexpr int src_b(int s) {
    int q = 0;
    for (int a = 0; a <= M - 2; ++a)
      for (int b = 0; a + b <= M - 2; ++b) {
        if (q == s) return b;
        ++q;
      }
    return -1;
  }
  __host__ __device__ static constexpr int src_of(int a, int b) {
    int q = 0;
    for (int aa = 0; aa <= M - 2; ++aa)
      for (int bb = 0; aa + bb <= M - 2; ++bb) {
        if (aa == a && bb == b) return q;
        ++q;
      }
    return -1;
  }

  __device__ static int wrap_fast(int i, int n, bool near) {
    if (near) return i < 0 ? i + n : (i >= n ? i - n : i);
    return wrap(i, n);
  }

  // a thread's share of a staged plane (the block has TXY^2 threads)
  static constexpr int kLoads = (kSu + TXY * TXY - 1) / (TXY * TXY);

  // loads of plane p (unwrapped index) into this thread's registers
  __device__ static void load_plane(const double* __restrict__ Uv, const Grid& g, int i0, int j0,
                                    int p, double (&r)[kLoads]) {
    const int k = wrap(p, g.nz);
    const bool nx_near = g.nx >= TXY + R, ny_near = g.ny >= TXY + R;
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
      const int e = threadIdx.x + l * TXY * TXY;
      if (e < kSu) {
        const int x = e % E, y = e / E;
        r[l] = Uv[zone_of(wrap_fast(i0 + x - R, g.nx, nx_near),
                          wrap_fast(j0 + y - R, g.ny, ny_near), k, g)];
      }
    }
  }

  // Stage plane p from this thread's registers cur, start the loads of
  // plane p+1 into next (when prefetch; they complete behind the sweeps),
  // then the x-y sweeps; ring slot of the plane; in-plane modes written to
  // W when write is set.
  __device__ static void plane_xy(const double* __restrict__ Uv, T* __restrict__ Wv, const Grid& g,
                                  int nvar, int i0, int j0, int p, bool write,
                                  const double (&cur)[kLoads], bool prefetch,
                                  double (&next)[kLoads], double* su, T* sx, double* ring0,
                                  T* ringT) {
    const int k = wrap(p, g.nz);
#pragma unroll
    for (int l = 0; l < kLoads; ++l) {
      const int e = threadIdx.x + l * TXY * TXY;
      if (e < kSu) su[e] = cur[l];
    }
    __syncthreads();
    if (prefetch) load_plane(Uv, g, i0, j0, p + 1, next);
    const int slot = ((p % NW) + NW) % NW;
    // x sweep on TXY x E lines: modes (a,0,0); the fields (a,0), a <= M-2,
    // of every row (the y sweep's input, y halo included)
    for (int e = threadIdx.x; e < TXY * E; e += blockDim.x) {
      const int x = e % TXY, y = e / TXY;
      const double* row = su + y * E + x;
      const double c = row[R];
      T d[2 * M - 1];
#pragma unroll
      for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(row[q] - c);
      T m[M];
      weno1d<T, M>(d, m);
#pragma unroll
      for (int a = 1; a <= M - 2; ++a) sx[((a - 1) * E + y) * TXY + x] = m[a];
      const bool inside = y >= R && y < R + TXY && i0 + x < g.nx && j0 + y - R < g.ny;
      if (write && inside) {
        const long long n = zone_of(i0 + x, j0 + y - R, k, g);
#pragma unroll
        for (int a = 1; a <= M - 1; ++a)
          Wv[(long long)(spatial_mode(a, 0, 0) - 1) * nvar * g.S + n] = m[a];
      }
      if (y >= R && y < R + TXY) {
        const int t = (y - R) * TXY + x;
        ring0[slot * TXY * TXY + t] = c;
#pragma unroll
        for (int a = 1; a <= M - 2; ++a)
          ringT[(slot * (NSRC - 1) + src_of(a, 0) - 1) * TXY * TXY + t] = m[a];
      }
    }
    __syncthreads();
    // y sweep on TXY x TXY lines of the fields (a,0), a <= M-2: (a,b,0)
    for (int t = threadIdx.x; t < TXY * TXY; t += blockDim.x) {
      const int x = t % TXY, y = t / TXY;
      const bool inside = i0 + x < g.nx && j0 + y < g.ny;
      const long long n = inside ? zone_of(i0 + x, j0 + y, k, g) : 0;
#pragma unroll
      for (int a = 0; a <= M - 2; ++a) {
        T d[2 * M - 1];
        if (a == 0) {
          const double c = su[(y + R) * E + x + R];
#pragma unroll
          for (int q = 0; q < 2 * M - 1; ++q) d[q] = T(su[(y + q) * E + x + R] - c);
        } else {
#pragma unroll
          for (int q = 0; q < 2 * M - 1; ++q) d[q] = sx[((a - 1) * E + y + q) * TXY + x];
        }
        T m[M];
        weno1d<T, M>(d, m);
#pragma unroll
        for (int bb = 1; bb <= M - 1 - a; ++bb) {
          if (write && inside) Wv[(long long)(spatial_mode(a, bb, 0) - 1) * nvar * g.S + n] = m[bb];
          if (a + bb <= M - 2)
            ringT[(slot * (NSRC - 1) + src_of(a, bb) - 1) * TXY * TXY + t] = m[bb];
        }
      }
    }
    // (the caller's next barrier orders these ring writes before the z sweep)
  }

  // z sweep of plane p (unwrapped, 0 <= p < nz): window p-R .. p+R in the ring
  __device__ static void plane_z(T* __restrict__ Wv, const Grid& g, int nvar, int i0, int j0,
                                 int p, const double* ring0, const T* ringT) {
    for (int t = threadIdx.x; t < TXY * TXY; t += blockDim.x) {
      const int x = t % TXY, y = t / TXY;
      if (!(i0 + x < g.nx && j0 + y < g.ny)) continue;
      const long long n = zone_of(i0 + x, j0 + y, p, g);
      int sl[NW];
#pragma unroll
      for (int q = 0; q < NW; ++q) sl[q] = (((p - R + q) % NW) + NW) % NW;
#pragma unroll
      for (int s = 0; s < NSRC; ++s) {
        const int a = src_a(s), b = src_b(s);
        T d[NW];
        if (s == 0) {
          const double c = ring0[sl[R] * TXY * TXY + t];
#pragma unroll
          for (int q = 0; q < NW; ++q) d[q] = T(ring0[sl[q] * TXY * TXY + t] - c);
        } else {
#pragma unroll
          for (int q = 0; q < NW; ++q) d[q] = ringT[(sl[q] * (NSRC - 1) + s - 1) * TXY * TXY + t];
        }
        T mo[M];
        weno1d<T, M>(d, mo);
#pragma unroll
        for (int c = 1; c <= M - 1 - a - b; ++c)
          Wv[(long long)(spatial_mode(a, b, c) - 1) * nvar * g.S + n] = mo[c];
      }
    }
  }

  // Planes k0 .. k1-1 of the column of tile (i0, j0) for one variable (Uv,
  // Wv: that variable's rows).  Planes k0-R .. k0+R-1 fill the ring first
  // (in-plane modes written for the segment's own planes); then for k = k0
  // .. k1-1 plane k+R is added (modes written while k+R < k1) and plane k's
  // z sweep runs, so every plane of the segment is written once.
  __device__ static void run(const double* __restrict__ Uv, T* __restrict__ Wv, const Grid& g,
                             int nvar, int i0, int j0, int k0, int k1, double* su, T* sx,
                             double* ring0, T* ringT) {
    double cur[kLoads], next[kLoads];
    load_plane(Uv, g, i0, j0, k0 - R, cur);
    for (int p = k0 - R; p < k0 + R; ++p) {
      plane_xy(Uv, Wv, g, nvar, i0, j0, p, p >= k0 && p < k1, cur, true, next, su, sx, ring0,
               ringT);
      __syncthreads();
#pragma unroll
      for (int l = 0; l < kLoads; ++l) cur[l] = next[l];
    }
    for (int k = k0; k < k1; ++k) {
      plane_xy(Uv, Wv, g, nvar, i0, j0, k + R, k + R < k1, cur, k + 1 < k1, next, su, sx, ring0,
               ringT);
      __syncthreads();
      // (the next plane's staging writes only su, and its ring writes come
      // after its first barrier, so this sweep's ring reads are done then)
      plane_z(Wv, g, nvar, i0, j0, k, ring0, ringT);
#pragma unroll
      for (int l = 0; l < kLoads; ++l) cur[l] = next[l];
    }
  }
};

// The z sweep along column segments: a thread takes the zones (i, j, k) of
// kZSeg consecutive planes and slides a window of 2M-1 planes down the
// column, so each source value is read once per segment (plus the 2(M-1)
// halo planes) instead of once per stencil point.  Same line reconstructions
// as weno_sweep_zone<.., 2, ..>: the sources are the moments (a, b, 0) with
// a + b <= M-2, the zone averages entering as differences in double.
constexpr int kZSeg = 8;

template <class T, int M, int NVAR>
struct ZColumn {
  static constexpr int R = M - 1, NW = 2 * R + 1;
  static constexpr int NSRC = M * (M - 1) / 2;   // sources (a, b) of the z sweep

  // source s -> (a, b) in the order of the sweep kernel's loops
  __host__ __device__ static constexpr int src_a(int s) {
    int q = 0;
    for (int a = 0; a <= M - 2; ++a)
      for (int b = 0; a + b <= M - 2; ++b) {
        if (q == s) return a;
        ++q;
      }
    return -1;
  }
  __host__ __device__ static constexpr int src_b(int s) {
    int q = 0;
    for (int a = 0; a <= M - 2; ++a)
      for (int b = 0; a + b <= M - 2; ++b) {
        if (q == s) return b;
        ++q;
      }
    return -1;
  }

  __device__ static void load(const double* __restrict__ U, const T* __restrict__ W, const Grid& g,
                              long long z, double (&u)[NVAR], T (&f)[NSRC > 1 ? NSRC - 1 : 1][NVAR]) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) u[v] = U[(long long)v * g.S + z];
#pragma unroll
    for (int s = 1; s < NSRC; ++s) {
      const int src = spatial_mode(src_a(s), src_b(s), 0);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) f[s - 1][v] = W[((long long)(src - 1) * NVAR + v) * g.S + z];
    }
  }

  // The window holds planes k-R .. k+R and one plane ahead (k+R+1), whose
  // loads are issued before plane k is reconstructed so that their latency
  // overlaps the arithmetic.
  __device__ static void run(const double* __restrict__ U, T* __restrict__ W, const Grid& g, int i,
                             int j, int k0, int k1) {
    double wu[NW + 1][NVAR];
    T wf[NW + 1][NSRC > 1 ? NSRC - 1 : 1][NVAR];
#pragma unroll
    for (int q = 0; q < NW; ++q)
      load(U, W, g, zone_of(i, j, wrap(k0 - R + q, g.nz), g), wu[q], wf[q]);
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
      if (k + 1 < k1) load(U, W, g, zone_of(i, j, wrap(k + R + 1, g.nz), g), wu[NW], wf[NW]);
      const long long n = zone_of(i, j, k, g);
#pragma unroll
      for (int s = 0; s < NSRC; ++s) {
        const int a = src_a(s), b = src_b(s);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          T d[NW];
#pragma unroll
          for (int q = 0; q < NW; ++q)
            d[q] = s == 0 ? T(wu[q][v] - wu[R][v]) : wf[q][s > 0 ? s - 1 : 0][v];
          T mo[M];
          weno1d<T, M>(d, mo);
#pragma unroll
          for (int c = 1; c <= M - 1 - a - b; ++c)
            W[((long long)(spatial_mode(a, b, c) - 1) * NVAR + v) * g.S + n] = mo[c];
        }
      }
#pragma unroll
      for (int q = 0; q < NW; ++q) {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) wu[q][v] = wu[q + 1][v];
#pragma unroll
        for (int s = 0; s < (NSRC > 1 ? NSRC - 1 : 1); ++s)
#pragma unroll
          for (int v = 0; v < NVAR; ++v) wf[q][s][v] = wf[q + 1][s][v];
      }
    }
  }
};

}  // namespace ader
