// Grouped ragged GEMM on the CDNA4 matrix cores.
//
// One launch runs many independent products C = beta*C + alpha*sum_s A_s B_s
// of different shapes (the level-synchronous GEMMs of the SMW updates,
// eq. (11), and the interpolation products of eq. (12) and
// the Skeletonize pass).  A product may have several K segments whose B
// operands live at unrelated addresses: that is how the solve's final
// product x = v - W~ e gathers the e blocks of a leaf's ancestors, and its
// W~ blocks of every level, without copying them.
//
// Tiles: 128 rows (four waves of 32 rows, each 2 x c MFMA 16x16x4 blocks,
// f64 or f32 accumulate) by 16 c columns, c <= 5 chosen per tile from the
// product's N, so skeleton-rank widths (32..80) waste at most 15 columns.
// K is staged through LDS in steps of 16, the next step's operands loaded
// into registers while the current one computes.
//
// Two output layouts.  C column-major: the MFMA takes the B fragment as its
// first operand, so 16 consecutive lanes hold 16 consecutive rows of C
// (coalesced column-major stores).  CT (C^T row-major, used when the
// planner transposes a product with few rows): the A fragment goes first and
// 16 consecutive lanes hold 16 consecutive columns.  Operand layout of both
// 16x16x4 forms: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element v of lane l is D[acc_row(l / 16, v)][l % 16].
#include "device_util.hpp"
#include "internal.hpp"

namespace invaskit {
namespace {

constexpr int BK = 16;
constexpr int GBM = kGemmTileM;    // 128
constexpr int GCB = kGemmMaxCols / 16;  // column blocks per tile, at most 5

template <typename T, bool CT>
__global__ __launch_bounds__(256) void k_gemm(const GemmProb* __restrict__ probs,
                                              const GemmSeg* __restrict__ segs,
                                              const Tile3* __restrict__ tiles) {
  using V4 = typename Vec4<T>::type;
  constexpr int BN = 16 * GCB;
  constexpr int NA = GBM * BK / 256;         // A elements per thread per K step
  constexpr int NB = (BN * BK + 255) / 256;  // B elements per thread per K step
  __shared__ T As[BK][GBM + 1];
  __shared__ T Bs[BK][BN + 1];

  const Tile3 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GemmProb P = probs[t.prob];
  const int m0 = t.tm * GBM;
  const int n0 = t.tn * kGemmColChunk;
  const int nw = (P.N <= kGemmMaxCols) ? P.N : min(kGemmColChunk, P.N - n0);  // tile width
  const int nc = (nw + 15) / 16;                                            // 1 .. GCB
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave * 32;
  const int lr = lane & 15;  // fragment row / column
  const int lk = lane >> 4;  // fragment k

  V4 acc[2][GCB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < GCB; ++j) acc[i][j] = V4{0, 0, 0, 0};

  // K steps run over the segments in order; the next step's operands are
  // loaded into registers while the current step computes from LDS
  T av[NA], bv[NB];
  int arm = 0;
  auto fetch = [&](const GemmSeg& g, int k0) {
    const gptr<const T> A = glb(static_cast<const T*>(g.A));
    const gptr<const T> B = glb(static_cast<const T*>(g.B));
    arm = g.a_rm;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int idx = tid + q * 256;
      const int i = arm ? idx / BK : idx % GBM;
      const int kk = arm ? idx % BK : idx / GBM;
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
      const int gk = k0 + kk;
      bv[q] = (j < nw && gk < g.k) ? B[(int64_t)(n0 + j) * g.ldb + gk] : T(0);
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
        As[idx / GBM][idx % GBM] = av[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int idx = tid + q * 256;
      if (idx < BN * BK) Bs[idx % BK][idx / BK] = bv[q];
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
      const T a0 = As[kk + lk][wm + lr];
      const T a1 = As[kk + lk][wm + 16 + lr];
#pragma unroll
      for (int j = 0; j < GCB; ++j) {
        if (j < nc) {
          const T b = Bs[kk + lk][16 * j + lr];
          if constexpr (CT) {
            acc[0][j] = mfma16(a0, b, acc[0][j]);
            acc[1][j] = mfma16(a1, b, acc[1][j]);
          } else {
            acc[0][j] = mfma16(b, a0, acc[0][j]);
            acc[1][j] = mfma16(b, a1, acc[1][j]);
          }
        }
      }
    }
  }

  const gptr<T> C = glb(static_cast<T*>(P.C));
  const T alpha = (T)P.alpha;
  const T beta = (T)P.beta;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < GCB; ++j) {
      if (j >= nc) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row, col;
        if constexpr (CT) {
          row = m0 + wm + 16 * i + acc_row(T(0), lk, v);
          col = 16 * j + lr;
        } else {
          row = m0 + wm + 16 * i + lr;
          col = 16 * j + acc_row(T(0), lk, v);
        }
        if (row < P.M && col < nw) {
          const gptr<T> c = CT ? C + (int64_t)row * P.ldc + n0 + col : C + (int64_t)(n0 + col) * P.ldc + row;
          const T r = alpha * acc[i][j][v];
          *c = (P.beta != 0.0) ? beta * (*c) + r : r;
        }
      }
    }
  }
}

// Calls f(std::integral_constant<int, NC>) with NC = n (1 .. kGemvCols): the
// skinny products' column loops get a compile-time trip count, so their
// loads carry no per-column branch (a load under a branch was waited for
// before the next one issued).
template <typename F>
__device__ __forceinline__ void with_cols(int n, F&& f) {
  switch (n) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: f(std::integral_constant<int, kGemvCols>{}); break;
  }
}

// Skinny products (N <= 4 columns, every A column-major, M <= 128): one
// workgroup per product.  The 256 threads cover R rows by 256 / R groups of
// K, R the smallest power of two (16 .. 128) not below M, so that short
// products (the solve's top-down pass: M = a skeleton rank, 32 .. 71) keep
// every lane busy; consecutive threads read consecutive rows of a column
// (coalesced), and the groups' partial sums are added through LDS in a fixed
// order.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv(const GemmProb* __restrict__ probs,
                                              const GemmSeg* __restrict__ segs) {
  __shared__ T part[256][kGemvCols];
  const GemmProb P = probs[blockIdx.x];
  const gptr<T> C = glb(static_cast<T*>(P.C));
  const int tid = threadIdx.x;
  const int R = P.M <= 16 ? 16 : P.M <= 32 ? 32 : P.M <= 64 ? 64 : 128;
  const int G = 256 / R;
  const int row = tid & (R - 1), kg = tid / R;
  const bool rin = row < P.M;
  T acc[kGemvCols];
#pragma unroll
  for (int c = 0; c < kGemvCols; ++c) acc[c] = T(0);
  with_cols(P.N, [&](auto NCc) {
    constexpr int NC = decltype(NCc)::value;
    for (int sg = P.seg0; sg < P.seg0 + P.nseg; ++sg) {
      const GemmSeg g = segs[sg];
      const gptr<const T> A = glb(static_cast<const T*>(g.A)) + (rin ? row : 0);
      const gptr<const T> B = glb(static_cast<const T*>(g.B));
#pragma unroll 8
      for (int k = kg; k < g.k; k += G) {
        const T a = A[(int64_t)k * g.lda];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fma(a, B[(int64_t)c * g.ldb + k], acc[c]);
      }
    }
  });
#pragma unroll
  for (int c = 0; c < kGemvCols; ++c) part[tid][c] = rin ? acc[c] : T(0);
  __syncthreads();
  if (tid < R && rin) {
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) {
      if (c < P.N) {
        T sum = part[tid][c];
        for (int q = 1; q < G; ++q) sum += part[q * R + tid][c];
        const gptr<T> out = C + (int64_t)c * P.ldc + tid;
        const T r = (T)P.alpha * sum;
        *out = (P.beta != 0.0) ? (T)P.beta * (*out) + r : r;
      }
    }
  }
}

// Skinny products (N <= 4, A column-major) taller than kGemvRows (the
// solve's final product x = v - W~ e, a leaf's rows against every level's
// W~ block): workgroups of kGemvTallRows = 256 rows from the tile list
// (product, row block).  Lane l takes rows 4 l .. 4 l + 3 (one 16-byte load
// per column in FP32, two in FP64) and the four waves split K; the waves'
// partial sums are added through LDS in a fixed order.  A row group that
// straddles the last row is read element by element, so no load passes the
// product's last row.  B is the same for every lane (a broadcast load).
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_tall(const GemmProb* __restrict__ probs,
                                                   const GemmSeg* __restrict__ segs,
                                                   const Tile3* __restrict__ tiles) {
  typedef T vec4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
  __shared__ T part[4][kGemvTallRows][kGemvCols];
  const Tile3 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GemmProb P = probs[t.prob];
  const gptr<T> C = glb(static_cast<T*>(P.C));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lrow = 4 * lane;                       // first of the lane's rows in the block
  const int row = t.tm * kGemvTallRows + lrow;     // in the product
  const int nr = max(0, min(4, P.M - row));        // rows of the group inside the product
  T acc[4][kGemvCols];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) acc[i][c] = T(0);
  with_cols(P.N, [&](auto NCc) {
    constexpr int NC = decltype(NCc)::value;
    for (int sg = P.seg0; sg < P.seg0 + P.nseg; ++sg) {
      const GemmSeg g = segs[sg];
      const gptr<const T> A = glb(static_cast<const T*>(g.A)) + (nr > 0 ? row : 0);
      const gptr<const T> B = glb(static_cast<const T*>(g.B));
#pragma unroll 4
      for (int k = wave; k < g.k; k += 4) {
        const gptr<const T> ak = A + (int64_t)k * g.lda;
        vec4 a;
        if (nr == 4) {
          a = *(gptr<const vec4>)ak;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = (i < nr) ? ak[i] : T(0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const T b = B[(int64_t)c * g.ldb + k];
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][c] = fma(a[i], b, acc[i][c]);
        }
      }
    }
  });
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) part[wave][lrow + i][c] = acc[i][c];
  __syncthreads();
  // thread t finishes row t of the block
  const int tr = threadIdx.x;
  const int orow = t.tm * kGemvTallRows + tr;
  if (orow < P.M) {
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) {
      if (c < P.N) {
        const T sum = (part[0][tr][c] + part[1][tr][c]) + (part[2][tr][c] + part[3][tr][c]);
        const gptr<T> out = C + (int64_t)c * P.ldc + orow;
        const T r = (T)P.alpha * sum;
        *out = (P.beta != 0.0) ? (T)P.beta * (*out) + r : r;
      }
    }
  }
}

// Skinny products with row-major A (the projections by P): one wave per
// output row, lanes striding along the row (coalesced) and a butterfly sum
// across the wave.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_rm(const GemmProb* __restrict__ probs,
                                                 const GemmSeg* __restrict__ segs) {
  const GemmProb P = probs[blockIdx.x];
  const gptr<T> C = glb(static_cast<T*>(P.C));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int row = wave; row < P.M; row += 4) {
    T acc[kGemvCols];
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) acc[c] = T(0);
    with_cols(P.N, [&](auto NCc) {
      constexpr int NC = decltype(NCc)::value;
      for (int sg = P.seg0; sg < P.seg0 + P.nseg; ++sg) {
        const GemmSeg g = segs[sg];
        const gptr<const T> A = glb(static_cast<const T*>(g.A)) + (int64_t)row * g.lda;
        const gptr<const T> B = glb(static_cast<const T*>(g.B));
#pragma unroll 4
        for (int k = lane; k < g.k; k += 64) {
          const T a = A[k];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] = fma(a, B[(int64_t)c * g.ldb + k], acc[c]);
        }
      }
    });
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c)
      if (c < P.N)
        for (int off = 32; off >= 1; off >>= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kGemvCols; ++c) {
        if (c < P.N) {
          const gptr<T> out = C + (int64_t)c * P.ldc + row;
          const T r = (T)P.alpha * acc[c];
          *out = (P.beta != 0.0) ? (T)P.beta * (*out) + r : r;
        }
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_gemv(const GemmProb* probs, const GemmSeg* segs, int count, int form,
                       hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (form == kGemvRowMajor)
    hipLaunchKernelGGL((k_gemv_rm<T>), dim3(count), dim3(256), 0, s, probs, segs);
  else
    hipLaunchKernelGGL((k_gemv<T>), dim3(count), dim3(256), 0, s, probs, segs);
  return hipGetLastError();
}
template hipError_t launch_gemv<double>(const GemmProb*, const GemmSeg*, int, int, hipStream_t);
template hipError_t launch_gemv<float>(const GemmProb*, const GemmSeg*, int, int, hipStream_t);

template <typename T>
hipError_t launch_gemv_tall(const GemmProb* probs, const GemmSeg* segs, const Tile3* tiles,
                            int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemv_tall<T>), dim3(ntiles), dim3(kGemvTallRows), 0, s, probs, segs,
                     tiles);
  return hipGetLastError();
}
template hipError_t launch_gemv_tall<double>(const GemmProb*, const GemmSeg*, const Tile3*, int,
                                             hipStream_t);
template hipError_t launch_gemv_tall<float>(const GemmProb*, const GemmSeg*, const Tile3*, int,
                                            hipStream_t);

template <typename T>
hipError_t launch_gemm(const GemmProb* probs, const GemmSeg* segs, const Tile3* tiles,
                       int ntiles, bool transposed, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (transposed)
    hipLaunchKernelGGL((k_gemm<T, true>), dim3(ntiles), dim3(256), 0, s, probs, segs, tiles);
  else
    hipLaunchKernelGGL((k_gemm<T, false>), dim3(ntiles), dim3(256), 0, s, probs, segs, tiles);
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmProb*, const GemmSeg*, const Tile3*, int, bool,
                                        hipStream_t);
template hipError_t launch_gemm<float>(const GemmProb*, const GemmSeg*, const Tile3*, int, bool,
                                       hipStream_t);

}  // namespace invaskit
