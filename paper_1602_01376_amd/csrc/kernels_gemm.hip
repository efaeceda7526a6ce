// Grouped ragged GEMM on the CDNA4 matrix cores.
//
// One launch runs many independent products C = beta*C + alpha*sum_s A_s B_s
// of different shapes (the level-synchronous GEMMs of the SMW updates,
// eq. (11), and the interpolation products of eq. (12) and
// the Skeletonize pass).  A product may have several K segments whose B
// operands live at unrelated addresses: that is how the deferred correction
// gathers the per-level y blocks of a leaf's ancestors without copying them.
//
// Tiles: BM x BN outputs per workgroup of 4 waves, each wave a 32 x 32 block
// computed as 2 x 2 MFMA 16x16x4 blocks (f64 or f32 accumulate).  Two shapes:
// 64 x 64, and 128 x 32 for products with at most 32 columns (the deferred
// corrections and skeleton projections, whose N is a skeleton rank).
// K is staged through LDS in steps of 16, the next step's operands loaded
// into registers while the current one computes.  The MFMA is issued with the B
// fragment as its first operand so that the accumulator layout puts 16
// consecutive lanes on 16 consecutive rows of column-major C (coalesced
// stores).  Operand layout of both 16x16x4 forms: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator element v of lane l
// is D[4 (l / 16) + v][l % 16] for f32 but D[l / 16 + 4 v][l % 16] for f64
// (measured on gfx950).
#include "internal.hpp"

namespace invaskit {
namespace {

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

// accumulator row of element v in lane group g = l / 16 (see above)
__device__ __forceinline__ constexpr int acc_row(double, int g, int v) { return g + 4 * v; }
__device__ __forceinline__ constexpr int acc_row(float, int g, int v) { return 4 * g + v; }

__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int BK = 16;
constexpr int PAD = 1;

template <typename T, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm(const GemmProb* __restrict__ probs,
                                              const GemmSeg* __restrict__ segs,
                                              const Tile3* __restrict__ tiles) {
  using V4 = typename Vec4<T>::type;
  constexpr int WN = BN / 32;              // waves along N
  constexpr int NA = BM * BK / 256;        // A elements per thread
  constexpr int NB = BN * BK / 256;        // B elements per thread
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  const Tile3 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GemmProb P = probs[t.prob];
  const int m0 = t.tm * BM;
  const int n0 = t.tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / WN) * 32;
  const int wn = (wave % WN) * 32;
  const int lr = lane & 15;  // fragment row / column
  const int lk = lane >> 4;  // fragment k

  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  // K steps run over the segments in order; the next step's operands are
  // loaded into registers while the current step computes from LDS
  T av[NA], bv[NB];
  int arm = 0;
  auto fetch = [&](const GemmSeg& g, int k0) {
    const T* __restrict__ A = static_cast<const T*>(g.A);
    const T* __restrict__ B = static_cast<const T*>(g.B);
    arm = g.a_rm;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int idx = tid + q * 256;
      const int i = arm ? idx / BK : idx % BM;
      const int kk = arm ? idx % BK : idx / BM;
      const int gi = m0 + i, gk = k0 + kk;
      T v = 0;
      if (gi < P.M && gk < g.k)
        v = arm ? A[(int64_t)gi * g.lda + gk] : A[(int64_t)gk * g.lda + gi];
      av[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int idx = tid + q * 256;
      const int kk = idx % BK;
      const int j = idx / BK;
      const int gj = n0 + j, gk = k0 + kk;
      bv[q] = (gj < P.N && gk < g.k) ? B[(int64_t)gj * g.ldb + gk] : T(0);
    }
  };
  const int send = P.seg0 + P.nseg;
  int s = P.seg0, k0 = 0;
  GemmSeg g;
  if (s < send) {
    g = segs[s];
    fetch(g, 0);
  }
  while (s < send) {
    __syncthreads();  // the previous step's LDS reads are done
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int idx = tid + q * 256;
      if (arm)
        As[idx % BK][idx / BK] = av[q];
      else
        As[idx / BM][idx % BM] = av[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int idx = tid + q * 256;
      Bs[idx % BK][idx / BK] = bv[q];
    }
    __syncthreads();
    k0 += BK;
    if (k0 >= g.k) {
      ++s;
      k0 = 0;
      if (s < send) g = segs[s];
    }
    if (s < send) fetch(g, k0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a0 = As[kk + lk][wm + lr];
      T a1 = As[kk + lk][wm + 16 + lr];
      T b0 = Bs[kk + lk][wn + lr];
      T b1 = Bs[kk + lk][wn + 16 + lr];
      acc[0][0] = mfma16(b0, a0, acc[0][0]);
      acc[0][1] = mfma16(b1, a0, acc[0][1]);
      acc[1][0] = mfma16(b0, a1, acc[1][0]);
      acc[1][1] = mfma16(b1, a1, acc[1][1]);
    }
  }

  // with the operands swapped, accumulator element v of lane l holds
  // C[base_m + (l & 15)][base_n + acc_row(l >> 4, v)]
  T* __restrict__ C = static_cast<T*>(P.C);
  const T alpha = (T)P.alpha;
  const T beta = (T)P.beta;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = m0 + wm + i * 16 + lr;
    if (row >= P.M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = n0 + wn + j * 16 + acc_row(T(0), lk, v);
        if (col < P.N) {
          T* c = C + (int64_t)col * P.ldc + row;
          const T r = alpha * acc[i][j][v];
          *c = (P.beta != 0.0) ? beta * (*c) + r : r;
        }
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_gemm(const GemmProb* probs, const GemmSeg* segs, const Tile3* tiles,
                       int ntiles, int shape, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (shape == kGemmNarrow)
    hipLaunchKernelGGL((k_gemm<T, 128, 32>), dim3(ntiles), dim3(256), 0, s, probs, segs, tiles);
  else
    hipLaunchKernelGGL((k_gemm<T, 64, 64>), dim3(ntiles), dim3(256), 0, s, probs, segs, tiles);
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmProb*, const GemmSeg*, const Tile3*, int, int,
                                        hipStream_t);
template hipError_t launch_gemm<float>(const GemmProb*, const GemmSeg*, const Tile3*, int, int,
                                       hipStream_t);

}  // namespace invaskit
