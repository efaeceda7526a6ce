// Batched multi-right-hand-side solves with LU factors of uneven order (the
// leaf solves of Algorithm 2 and the reduced-system solves of eq.
// (e:blocksmw)), every system of a launch in one grid.
//
// One workgroup (4 waves) takes RT right-hand-side columns of one system.
// The permuted right-hand sides live in LDS (row-major, RT values per row).
// Forward substitution with the unit-lower L and back substitution with U
// proceed by 64-row blocks:
//   diagonal block: the 64 x 64 triangle is staged in LDS; each wave solves
//     RT/4 columns with lane = row, the finished value of row j broadcast by
//     a cross-lane read (no workgroup barrier inside the block);
//   off-diagonal update: the rows below (above) the block are updated on the
//     matrix cores, X_rows -= L[rows, block] X[block], in 16 x 16 tiles with
//     K = 64; the L operand streams from global memory, the solved block
//     rows from LDS.
// TZ is the type of the factors and of the arithmetic, TV the type of the
// right-hand sides in memory.  KIND only separates the kernel names of the
// three uses (leaf panels of the factorization, reduced systems, solve).
#include "internal.hpp"

namespace invaskit {
namespace {

constexpr int NBK = 64;  // row block

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  using type = f64x4;
};
template <>
struct Vec4<float> {
  using type = f32x4;
};
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// accumulator row of element v in lane group g = lane / 16 (16x16x4 forms,
// measured on gfx950): f32 4g + v, f64 g + 4v.  Column = lane % 16.
__device__ __forceinline__ constexpr int acc_row(double, int g, int v) { return g + 4 * v; }
__device__ __forceinline__ constexpr int acc_row(float, int g, int v) { return 4 * g + v; }

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <typename TZ>
constexpr int cols_per_tile() {
  return sizeof(TZ) == 8 ? 16 : 32;
}

template <typename TZ, typename TV, int KIND>
__global__ __launch_bounds__(256) void k_getrs(const TrsmProb* __restrict__ probs,
                                               const Tile2* __restrict__ tiles) {
  using V4 = typename Vec4<TZ>::type;
  constexpr int RT = cols_per_tile<TZ>();
  constexpr int CW = RT / 4;  // columns per wave in the diagonal solve
  constexpr int CT = RT / 16; // 16-wide column tiles in the update
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
  const int lr = lane & 15, lk = lane >> 4;

  extern __shared__ __align__(16) unsigned char smem[];
  TZ* Ld = reinterpret_cast<TZ*>(smem);  // 64 x 64 diagonal block, column-major
  TZ* X = Ld + NBK * NBK;                // n x RT, row-major

  // gather the permuted right-hand sides: one thread per row, all RT column
  // loads of a row in flight together
  for (int i = tid; i < n; i += 256) {
    const int src = pr.perm[i];
    const TV* base = (src < pr.split) ? in0 + src : in1 + (src - pr.split);
    const int64_t ld = (src < pr.split) ? pr.ldin0 : pr.ldin1;
    TZ v[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) v[c] = (c < nc) ? (TZ)base[(int64_t)(c0 + c) * ld] : TZ(0);
#pragma unroll
    for (int c = 0; c < RT; ++c) X[i * RT + c] = v[c];
  }

  const int nblocks = (n + NBK - 1) / NBK;
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int bi = 0; bi < nblocks; ++bi) {
      const int b = fwd ? bi : nblocks - 1 - bi;
      const int jb = b * NBK;
      const int nb = min(NBK, n - jb);
      // stage the diagonal block
#pragma unroll
      for (int idx = tid; idx < NBK * NBK; idx += 256) {
        const int r = idx % NBK, j = idx / NBK;
        Ld[idx] = (r < nb && j < nb) ? LU[(int64_t)(jb + j) * n + jb + r] : TZ(0);
      }
      __syncthreads();
      {
        const int r = jb + lane;
        TZ x[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) x[q] = (lane < nb) ? X[r * RT + wave * CW + q] : TZ(0);
        if (fwd) {
          for (int j = 0; j < nb - 1; ++j) {
            const TZ l = (lane > j) ? Ld[j * NBK + lane] : TZ(0);
#pragma unroll
            for (int q = 0; q < CW; ++q) x[q] -= l * lane_bcast(x[q], j);
          }
        } else {
          for (int j = nb - 1; j >= 0; --j) {
            const TZ u = (lane <= j) ? Ld[j * NBK + lane] : TZ(1);
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
        }
        if (lane < nb) {
#pragma unroll
          for (int q = 0; q < CW; ++q) X[r * RT + wave * CW + q] = x[q];
        }
      }
      __syncthreads();
      // off-diagonal update on the matrix cores: one 16-row tile per item,
      // its 16 x 64 slice of the factor loaded into registers up front
      const int r0 = fwd ? jb + nb : 0;
      const int r1 = fwd ? n : jb;
      const int nrt = (r1 - r0 + 15) / 16;
      for (int item = wave; item < nrt; item += 4) {
        const int row = r0 + item * 16 + lr;
        const bool rin = row < r1;
        TZ a[NBK / 4];
#pragma unroll
        for (int q = 0; q < NBK / 4; ++q) {
          const int j = 4 * q + lk;
          a[q] = (rin && j < nb) ? LU[(int64_t)(jb + j) * n + row] : TZ(0);
        }
        V4 acc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = V4{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NBK / 4; ++q) {
          const int j = 4 * q + lk;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const TZ bb = (j < nb) ? X[(jb + j) * RT + ct * 16 + lr] : TZ(0);
            acc[ct] = mfma16(a[q], bb, acc[ct]);
          }
        }
        const int i0 = r0 + item * 16;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = i0 + acc_row(TZ(0), lk, v);
            if (rr < r1) X[rr * RT + ct * 16 + lr] -= acc[ct][v];
          }
      }
      __syncthreads();
    }
  }

  for (int i = tid; i < n; i += 256) {
#pragma unroll
    for (int c = 0; c < RT; ++c)
      if (c < nc) out[(int64_t)(c0 + c) * pr.ldout + i] = (TV)X[i * RT + c];
  }
}

template <typename TZ, typename TV, int KIND>
hipError_t run(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, hipStream_t s) {
  constexpr int RT = cols_per_tile<TZ>();
  const size_t sm = ((size_t)NBK * NBK + (size_t)nmax * RT) * sizeof(TZ);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrs<TZ, TV, KIND>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_getrs<TZ, TV, KIND>), dim3(ntiles), dim3(256), sm, s, probs, tiles);
  return hipGetLastError();
}

}  // namespace

int getrs_cols_per_tile(bool tz64) { return tz64 ? cols_per_tile<double>() : cols_per_tile<float>(); }

template <typename TZ, typename TV>
hipError_t launch_getrs(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, int kind,
                        hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (kind) {
    case 0: return run<TZ, TV, 0>(probs, tiles, ntiles, nmax, s);
    case 1: return run<TZ, TV, 1>(probs, tiles, ntiles, nmax, s);
    default: return run<TZ, TV, 2>(probs, tiles, ntiles, nmax, s);
  }
}

template hipError_t launch_getrs<double, double>(const TrsmProb*, const Tile2*, int, int, int,
                                                 hipStream_t);
template hipError_t launch_getrs<float, float>(const TrsmProb*, const Tile2*, int, int, int,
                                               hipStream_t);
template hipError_t launch_getrs<double, float>(const TrsmProb*, const Tile2*, int, int, int,
                                                hipStream_t);

}  // namespace invaskit
