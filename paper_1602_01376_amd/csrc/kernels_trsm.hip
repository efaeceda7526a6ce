// Batched multi-right-hand-side solves with LU factors of uneven order (the
// leaf solves of Algorithm 2 and the reduced-system solves of eq.
// (11)), every system of a launch in one grid.
//
// Factors are stored row-major as the batched LU writes them: logical row j
// of the packed L\U sits in physical row perm[j], so every factor row is
// read through perm.
//
// k_diag_inv runs once per factorization: for every 64 x 64 diagonal block
// of every factor it forms the inverses of the unit-lower block of L and of
// the upper block of U (one wave each, one column of the inverse per lane,
// the diagonal of U inverted once), stored row-major.
//
// k_getrs: one workgroup (4 waves) takes 16 CT right-hand-side columns of
// one system (CT = 1 or 2); the permuted right-hand sides live in LDS (row
// stride 16 CT + 1 to spread the banks).  At CT = 2 every factor tile read
// serves two 16-column MFMA tiles, for twice the LDS per workgroup.  Forward substitution with L and back substitution with U go
// by 64-row blocks, both steps on the matrix cores:
//   diagonal block:  X_b = inv(L_bb) X_b   (inv(U_bb) going back),
//   off-diagonal:    X_rows -= L[rows, block] X_b   (U[rows, block] going back),
// in 16 x 16 output tiles with K = 64, the factor operands streamed from
// global memory as 16-byte row segments (see load_row_sigma).
// TZ is the type of the factors and of the arithmetic, TV the type of the
// right-hand sides in memory.  KIND 0..2 separate the kernel names of the
// library's three uses (leaf panels of the factorization, reduced systems,
// solve); their factor storage is padded by 64 elements, so a factor row is
// always read as whole 16-byte vectors, masked past the block's last column
// (no divergent paths that would drain the loads issued ahead).  KIND 3
// reads caller-owned factors and never touches memory past a row's block.
#include "device_util.hpp"
#include "internal.hpp"

namespace invaskit {
namespace {

constexpr int NBK = kDiagBlock;  // 64-row block

// ------------------------------------------------------------ block inverses
// Two waves per block, lane = column c of the inverse: wave 0 solves
// L x = e_c (unit lower, forward), wave 1 U x = e_c (backward, the diagonal
// of U inverted once).  Each lane keeps its whole column in registers and
// substitutes column-oriented: once x_k is final, x_i -= F[i][k] x_k for the
// rest, with F[.][k] read from LDS at one address for the whole wave (a
// broadcast).  No value crosses lanes, so the 64 steps are a chain of
// independent FMAs rather than of cross-lane broadcasts.
constexpr int DIP = NBK + 4;  // LDS row stride: 16-byte aligned rows

template <typename TZ>
__global__ __launch_bounds__(128, 2) void k_diag_inv(const DiagInvProb* __restrict__ probs) {
  const DiagInvProb p = probs[blockIdx.x];
  const gptr<const TZ> LU = glb(static_cast<const TZ*>(p.lu));
  const gptr<const int32_t> perm = glb(p.perm);
  const gptr<TZ> out = glb(static_cast<TZ*>(p.out));  // inv(L_bb) then inv(U_bb), 64 x 64 each
  const int n = p.n, jb = p.jb;
  const int nb = min(NBK, n - jb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ __align__(16) TZ B[NBK][DIP];  // B[k][i] = block entry (row i, column k)
  __shared__ TZ rdiag[NBK];
  __shared__ int s_perm[NBK];
  if (tid < NBK) s_perm[tid] = perm[jb + min(tid, nb - 1)];
  __syncthreads();
  // consecutive threads read consecutive columns of a factor row; all 32
  // loads of a thread are issued before any is stored (indices past the
  // block read its last row or column and are zeroed)
  constexpr int PER = NBK * NBK / 128;
  TZ v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + 128 * q;
    const int k = idx % NBK, i = idx / NBK;
    v[q] = LU[(int64_t)s_perm[min(i, nb - 1)] * n + jb + min(k, nb - 1)];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + 128 * q;
    const int k = idx % NBK, i = idx / NBK;
    B[k][i] = (i < nb && k < nb) ? v[q] : TZ(0);
  }
  __syncthreads();
  if (tid < NBK) rdiag[tid] = (tid < nb) ? TZ(1) / B[tid][tid] : TZ(0);
  __syncthreads();
  const int c = lane;
  TZ x[NBK];
#pragma unroll
  for (int i = 0; i < NBK; ++i) x[i] = (i == c && c < nb) ? TZ(1) : TZ(0);
  if (wave == 0) {
    // inv(L): forward, L unit lower
#pragma unroll
    for (int k = 0; k < NBK - 1; ++k) {
      const TZ xk = x[k];
#pragma unroll
      for (int i = k + 1; i < NBK; ++i) x[i] -= B[k][i] * xk;
    }
  } else {
    // inv(U): backward
#pragma unroll
    for (int k = NBK - 1; k >= 0; --k) {
      x[k] *= rdiag[k];
      const TZ xk = x[k];
#pragma unroll
      for (int i = 0; i < k; ++i) x[i] -= B[k][i] * xk;
    }
  }
  const gptr<TZ> dst = out + wave * NBK * NBK;  // row-major: lanes of a row store consecutive columns
#pragma unroll
  for (int i = 0; i < NBK; ++i) dst[i * NBK + c] = (i < nb && c < nb) ? x[i] : TZ(0);
}

// ------------------------------------------------------------------- solves
template <typename TZ, typename TV, int KIND, int CT>
__global__ __launch_bounds__(256) void k_getrs(const TrsmProb* __restrict__ probs,
                                               const Tile2* __restrict__ tiles) {
  using V4 = typename Vec4<TZ>::type;
  constexpr int RT = 16 * CT;  // right-hand sides of the workgroup
  constexpr int RTP = RT + 1;  // LDS row stride
  const Tile2 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const TrsmProb pr = probs[t.prob];
  const int n = pr.n;
  const int c0 = t.tn * RT;
  const int nc = min(RT, pr.nrhs - c0);
  const gptr<const TZ> LU = glb(static_cast<const TZ*>(pr.lu));
  const gptr<const TZ> DI = glb(static_cast<const TZ*>(pr.dinv));
  const gptr<const TV> in0 = glb(static_cast<const TV*>(pr.in0));
  const gptr<const TV> in1 = glb(static_cast<const TV*>(pr.in1));
  const gptr<const int32_t> perm = glb(pr.perm);
  const gptr<TV> out = glb(static_cast<TV*>(pr.out));
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the wave index is uniform: kept in a scalar register, the item loops
  // below branch on scalars and their loads need no divergent paths
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lg = lane >> 4;

  extern __shared__ __align__(16) unsigned char smem[];
  TZ* X = reinterpret_cast<TZ*>(smem);  // n x RT, row stride RTP
  int* Pm = reinterpret_cast<int*>(smem + (size_t)n * RTP * sizeof(TZ));  // perm, n entries

  // Block steps q = 0 .. 2 nblocks - 1: forward substitution over the blocks,
  // then back substitution in reverse.  Factor data never depends on X, so
  // the next step's inverse diagonal rows and each step's first off-diagonal
  // tile are loaded ahead of the barriers that separate the steps.
  const int nblocks = (n + NBK - 1) / NBK;
  const int nsteps = 2 * nblocks;
  TZ da[NBK / 4];  // this wave's 16 rows of the current step's diagonal inverse
  auto load_d = [&](int q) {
    const bool f = q < nblocks;
    const int bq = f ? q : nsteps - 1 - q;
    const gptr<const TZ> D = DI + (int64_t)(2 * bq + (f ? 0 : 1)) * NBK * NBK;
    load_row_sigma_raw(D + (16 * wave + lr) * NBK, lg, da);
  };
  load_d(0);

  // gather the permuted right-hand sides: one thread per row, 16 column
  // loads of the row in flight together (columns past the last read the
  // last one again and are zeroed)
  for (int i = tid; i < n; i += 256) {
    const int src = perm[i];
    Pm[i] = src;
    const gptr<const TV> base = (src < pr.split) ? in0 + src : in1 + (src - pr.split);
    const int64_t ld = (src < pr.split) ? pr.ldin0 : pr.ldin1;
#pragma unroll 1
    for (int ct = 0; ct < CT; ++ct) {
      TZ v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const TZ e = (TZ)base[(int64_t)(c0 + min(16 * ct + c, nc - 1)) * ld];
        v[c] = (16 * ct + c < nc) ? e : TZ(0);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) X[i * RTP + 16 * ct + c] = v[c];
    }
  }
  __syncthreads();

  for (int q = 0; q < nsteps; ++q) {
    const bool fwd = q < nblocks;
    const int b = fwd ? q : nsteps - 1 - q;
    const int jb = b * NBK;
    const int nb = min(NBK, n - jb);
    // rows below (above) the block, updated after the diagonal step
    const int r0 = fwd ? jb + nb : 0;
    const int r1 = fwd ? n : jb;
    const int nrt = (r1 - r0 + 15) / 16;
    // factor rows of one 16-row item.  Rows past r1 read row r1 - 1 (their
    // products are discarded); the library's factors are padded by one
    // block, so whole segments are read and the part past the block is
    // zeroed where it is used (KIND 3 reads only inside the block).
    auto load_f = [&](int item, TZ (&a)[NBK / 4]) {
      const int row = r0 + item * 16 + lr;
      const gptr<const TZ> rowp = LU + (int64_t)Pm[min(row, r1 - 1)] * n + jb;
      if constexpr (KIND == 3)
        load_row_sigma_g(rowp, row < r1 ? nb : 0, lg, a);
      else
        load_row_sigma_raw(rowp, lg, a);
    };
    TZ fa[NBK / 4], fb[NBK / 4];
    if (nrt > 0) load_f(min(wave, nrt - 1), fa);
    // X_b = inv(diagonal block) X_b: wave w computes rows 16w .. 16w+15 of
    // each 16-column tile
    {
      // every column tile's LDS reads are issued before the first product
      // (the scheduling barrier keeps the compiler from sinking each read
      // next to its product, which serialized the reads' latencies)
      TZ bb[CT][NBK / 4];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int kk = 0; kk < NBK / 4; ++kk) {
          const int k = sigma_k<TZ>(kk, lg);
          const TZ v = X[min(jb + k, n - 1) * RTP + 16 * ct + lr];
          bb[ct][kk] = (k < nb) ? v : TZ(0);
        }
      __builtin_amdgcn_sched_barrier(0);
      V4 acc[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        acc[ct] = V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NBK / 4; ++kk) acc[ct] = mfma16(da[kk], bb[ct][kk], acc[ct]);
      }
      __syncthreads();
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * wave + acc_row(TZ(0), lg, v);
          if (r < nb) X[(jb + r) * RTP + 16 * ct + lr] = acc[ct][v];
        }
    }
    __syncthreads();
    if (q + 1 < nsteps) load_d(q + 1);
    // X_rows -= F[rows, block] X_b.  X_b is not written here, so its MFMA
    // operands are read once; the next tile's factor rows are in flight
    // while the current one computes, and each factor tile serves all CT
    // column tiles.
    TZ xb[CT][NBK / 4];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int kk = 0; kk < NBK / 4; ++kk) {
        const int j = sigma_k<TZ>(kk, lg);
        const TZ v = X[min(jb + j, n - 1) * RTP + 16 * ct + lr];
        xb[ct][kk] = (j < nb) ? v : TZ(0);
      }
    auto update = [&](int item, TZ (&a)[NBK / 4]) {
      const int i0 = r0 + item * 16;
      // the item's rows are this wave's alone in this step: read them
      // before the products so the LDS latency overlaps them
      TZ xo[CT][4];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          xo[ct][v] = X[min(i0 + acc_row(TZ(0), lg, v), r1 - 1) * RTP + 16 * ct + lr];
      if (KIND != 3 && nb < NBK) mask_sigma(nb, lg, a);
      V4 acc[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        acc[ct] = V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NBK / 4; ++kk) acc[ct] = mfma16(a[kk], xb[ct][kk], acc[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = i0 + acc_row(TZ(0), lg, v);
          if (rr < r1) X[rr * RTP + 16 * ct + lr] = xo[ct][v] - acc[ct][v];
        }
    };
    // loads past the last item re-read it (no branch around a load)
    for (int item = wave; item < nrt; item += 8) {
      load_f(min(item + 4, nrt - 1), fb);
      update(item, fa);
      load_f(min(item + 8, nrt - 1), fa);
      if (item + 4 < nrt) update(item + 4, fb);
    }
    __syncthreads();
  }

  for (int i = tid; i < n; i += 256) {
#pragma unroll 1
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (16 * ct + c < nc)
          out[(int64_t)(c0 + 16 * ct + c) * pr.ldout + i] = (TV)X[i * RTP + 16 * ct + c];
  }
}

template <typename TZ, typename TV, int KIND, int CT>
hipError_t run(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, hipStream_t s) {
  const size_t sm = getrs_lds_bytes(nmax, sizeof(TZ), 16 * CT);
  if (sm > (size_t)kLdsBytes) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrs<TZ, TV, KIND, CT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_getrs<TZ, TV, KIND, CT>), dim3(ntiles), dim3(256), sm, s, probs, tiles);
  return hipGetLastError();
}

template <typename TZ, typename TV, int KIND>
hipError_t run_ct(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, int cols,
                  hipStream_t s) {
  if (cols == 32) return run<TZ, TV, KIND, 2>(probs, tiles, ntiles, nmax, s);
  if (cols == 16) return run<TZ, TV, KIND, 1>(probs, tiles, ntiles, nmax, s);
  return hipErrorInvalidValue;
}

}  // namespace

size_t getrs_lds_bytes(int nmax, size_t tz_bytes, int cols) {
  return (size_t)nmax * ((cols + 1) * tz_bytes + sizeof(int));
}

template <typename TZ>
hipError_t launch_diag_inv(const DiagInvProb* probs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_diag_inv<TZ>), dim3(count), dim3(128), 0, s, probs);
  return hipGetLastError();
}

template <typename TZ, typename TV>
hipError_t launch_getrs(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, int kind,
                        int cols, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (kind) {
    case 0: return run_ct<TZ, TV, 0>(probs, tiles, ntiles, nmax, cols, s);
    case 1: return run_ct<TZ, TV, 1>(probs, tiles, ntiles, nmax, cols, s);
    case 2: return run_ct<TZ, TV, 2>(probs, tiles, ntiles, nmax, cols, s);
    default: return run_ct<TZ, TV, 3>(probs, tiles, ntiles, nmax, cols, s);
  }
}

template hipError_t launch_diag_inv<double>(const DiagInvProb*, int, hipStream_t);
template hipError_t launch_diag_inv<float>(const DiagInvProb*, int, hipStream_t);
template hipError_t launch_getrs<double, double>(const TrsmProb*, const Tile2*, int, int, int,
                                                 int, hipStream_t);
template hipError_t launch_getrs<float, float>(const TrsmProb*, const Tile2*, int, int, int, int,
                                               hipStream_t);
template hipError_t launch_getrs<double, float>(const TrsmProb*, const Tile2*, int, int, int, int,
                                                hipStream_t);

}  // namespace invaskit
