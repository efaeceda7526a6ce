// Batched multi-right-hand-side solves with LU factors of uneven order (the
// leaf solves of Algorithm 2 and the reduced-system solves of eq.
// (e:blocksmw)), all systems of a level in one launch.
//
// One workgroup takes RT right-hand-side columns of one system.  The
// permuted right-hand sides are staged in LDS (row-major, RT values per
// row, so that a row is read with broadcast vector loads).  Forward
// substitution with the unit-lower L and back substitution with U are
// blocked by 64 rows:
//   diagonal block: each wave solves RT/4 columns, lane = row, the solved
//     value of row j is broadcast with a cross-lane read (no workgroup
//     barrier inside the block);
//   off-diagonal update: every thread owns rows below (above) the block and
//     accumulates RT dot products against the block's solved rows.
// TZ is the type of the factors and of the arithmetic, TV the type of the
// right-hand sides in memory (FP32 vectors can be solved with FP64 factors).
#include "internal.hpp"

namespace invaskit {
namespace {

constexpr int RT = 16;   // right-hand sides per workgroup
constexpr int NBK = 64;  // row block

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <typename TZ, typename TV>
__global__ __launch_bounds__(256) void k_getrs(const TrsmProb* __restrict__ probs,
                                               const Tile2* __restrict__ tiles) {
  const Tile2 t = tiles[blockIdx.x];
  const TrsmProb pr = probs[t.prob];
  const int n = pr.n;
  const int c0 = t.tn * RT;
  const int nc = min(RT, pr.nrhs - c0);
  const TZ* __restrict__ LU = static_cast<const TZ*>(pr.lu);
  const TV* __restrict__ in0 = static_cast<const TV*>(pr.in0);
  const TV* __restrict__ in1 = static_cast<const TV*>(pr.in1);
  TV* __restrict__ out = static_cast<TV*>(pr.out);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int CW = RT / 4;  // columns per wave in the diagonal solve

  extern __shared__ __align__(16) unsigned char smem[];
  TZ* X = reinterpret_cast<TZ*>(smem);  // n x RT, row-major

  for (int idx = tid; idx < n * RT; idx += 256) {
    const int i = idx % n, c = idx / n;
    TZ v = 0;
    if (c < nc) {
      const int src = pr.perm[i];
      v = (src < pr.split) ? (TZ)in0[(int64_t)(c0 + c) * pr.ldin0 + src]
                           : (TZ)in1[(int64_t)(c0 + c) * pr.ldin1 + (src - pr.split)];
    }
    X[i * RT + c] = v;
  }
  __syncthreads();

  // ---------------- forward: L y = P b, L unit lower
  for (int jb = 0; jb < n; jb += NBK) {
    const int nb = min(NBK, n - jb);
    {
      const int r = jb + lane;
      TZ x[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) x[q] = (lane < nb) ? X[r * RT + wave * CW + q] : TZ(0);
      for (int j = 0; j < nb - 1; ++j) {
        const TZ l = (lane > j && lane < nb) ? LU[(int64_t)(jb + j) * n + r] : TZ(0);
#pragma unroll
        for (int q = 0; q < CW; ++q) x[q] -= l * lane_bcast(x[q], j);
      }
      if (lane < nb) {
#pragma unroll
        for (int q = 0; q < CW; ++q) X[r * RT + wave * CW + q] = x[q];
      }
    }
    __syncthreads();
    for (int i = jb + nb + tid; i < n; i += 256) {
      TZ acc[RT];
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = 0;
      for (int j = 0; j < nb; ++j) {
        const TZ l = LU[(int64_t)(jb + j) * n + i];
        const TZ* xr = X + (jb + j) * RT;
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] += l * xr[c];
      }
#pragma unroll
      for (int c = 0; c < RT; ++c) X[i * RT + c] -= acc[c];
    }
    __syncthreads();
  }

  // ---------------- backward: U x = y
  const int nblocks = (n + NBK - 1) / NBK;
  for (int b = nblocks - 1; b >= 0; --b) {
    const int jb = b * NBK;
    const int nb = min(NBK, n - jb);
    {
      const int r = jb + lane;
      TZ x[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) x[q] = (lane < nb) ? X[r * RT + wave * CW + q] : TZ(0);
      for (int j = nb - 1; j >= 0; --j) {
        const TZ u = (lane <= j) ? LU[(int64_t)(jb + j) * n + r] : TZ(1);
        // lane j finishes its row, then every lane above it is updated
        if (lane == j) {
#pragma unroll
          for (int q = 0; q < CW; ++q) x[q] /= u;
        }
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const TZ xj = lane_bcast(x[q], j);
          if (lane < j) x[q] -= u * xj;
        }
      }
      if (lane < nb) {
#pragma unroll
        for (int q = 0; q < CW; ++q) X[r * RT + wave * CW + q] = x[q];
      }
    }
    __syncthreads();
    for (int i = tid; i < jb; i += 256) {
      TZ acc[RT];
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = 0;
      for (int j = 0; j < nb; ++j) {
        const TZ u = LU[(int64_t)(jb + j) * n + i];
        const TZ* xr = X + (jb + j) * RT;
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] += u * xr[c];
      }
#pragma unroll
      for (int c = 0; c < RT; ++c) X[i * RT + c] -= acc[c];
    }
    __syncthreads();
  }

  for (int idx = tid; idx < n * nc; idx += 256) {
    const int i = idx % n, c = idx / n;
    out[(int64_t)(c0 + c) * pr.ldout + i] = (TV)X[i * RT + c];
  }
}

}  // namespace

int getrs_cols_per_tile() { return RT; }

template <typename TZ, typename TV>
hipError_t launch_getrs(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t sm = (size_t)nmax * RT * sizeof(TZ);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrs<TZ, TV>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_getrs<TZ, TV>), dim3(ntiles), dim3(256), sm, s, probs, tiles);
  return hipGetLastError();
}

template hipError_t launch_getrs<double, double>(const TrsmProb*, const Tile2*, int, int,
                                                 hipStream_t);
template hipError_t launch_getrs<float, float>(const TrsmProb*, const Tile2*, int, int,
                                               hipStream_t);
template hipError_t launch_getrs<double, float>(const TrsmProb*, const Tile2*, int, int,
                                                hipStream_t);

}  // namespace invaskit
