// Batched LU with partial pivoting for square matrices of uneven order, one
// workgroup per matrix, all matrices of a tree level in one launch (the leaf
// LU of Algorithm 1 and the LU of the reduced systems of eq. (e:blocksmw)).
//
// Right-looking blocked algorithm with panel width NB:
//   1. the panel (rows j0..n, NB columns) is loaded into LDS and factored
//      column by column; the pivot is the first row of largest magnitude
//      (LAPACK getrf semantics), found by a wavefront max-reduction
//      followed by a cross-wave reduction through LDS;
//   2. the panel's row interchanges, composed into one permutation of the
//      touched rows, are applied to the other columns (independent loads);
//   3. U12 = L11^-1 A12 (one thread per column) is written to global memory
//      and kept in LDS;
//   4. the trailing matrix is updated, A22 -= L21 U12, with 4 x 4 register
//      blocks fed from LDS.
// The row permutation is returned as perm[j] = original row now at row j;
// info = j+1 for the first zero or non-finite pivot in column j (the
// factorization continues without dividing, as LAPACK does).
#include <cmath>

#include "internal.hpp"

namespace invaskit {
namespace {

template <typename T>
__device__ __forceinline__ bool better(T v, int i, T bv, int bi) {
  // larger magnitude wins; ties go to the smaller row index
  return (v > bv) || (v == bv && i < bi);
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_getrf(const LuProb* __restrict__ probs) {
  const LuProb pr = probs[blockIdx.x];
  T* __restrict__ A = static_cast<T*>(pr.a);
  const int n = pr.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  extern __shared__ __align__(16) unsigned char smem[];
  T* Pn = reinterpret_cast<T*>(smem);           // panel, (n - j0) x NB, ld = n - j0
  T* Us = Pn + (size_t)n * NB;                    // U12, NB x n, row-major (ld n)
  int* Ps = reinterpret_cast<int*>(Us + (size_t)NB * n);  // permutation
  int* Loc = Ps + n;  // composed interchanges of one panel
  __shared__ T red_v[4];
  __shared__ int red_i[4];
  __shared__ int s_piv[NB];
  __shared__ int s_tl[2 * NB];
  __shared__ int s_cnt;
  __shared__ int s_info;

  for (int i = tid; i < n; i += 256) Ps[i] = i;
  if (tid == 0) s_info = 0;
  __syncthreads();

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = min(NB, n - j0);
    const int mr = n - j0;  // panel rows
    for (int idx = tid; idx < mr * jb; idx += 256) {
      const int r = idx % mr, c = idx / mr;
      Pn[r + c * mr] = A[(int64_t)(j0 + c) * n + j0 + r];
    }
    __syncthreads();

    for (int jj = 0; jj < jb; ++jj) {
      // ---- pivot search in column jj, rows jj..mr
      T bv = T(-1);
      int bi = 0x7fffffff;
      for (int r = jj + tid; r < mr; r += 256) {
        const T v = fabs(Pn[r + jj * mr]);
        const T vv = (v == v) ? v : T(INFINITY);  // a NaN is taken as pivot (flagged below)
        if (better(vv, r, bv, bi)) {
          bv = vv;
          bi = r;
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const T ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (better(ov, oi, bv, bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_v[wave] = bv;
        red_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        T v = red_v[0];
        int i = red_i[0];
        for (int w = 1; w < 4; ++w)
          if (better(red_v[w], red_i[w], v, i)) {
            v = red_v[w];
            i = red_i[w];
          }
        s_piv[jj] = i;
        const int p = i;
        // swap the permutation entries
        const int a = Ps[j0 + jj];
        Ps[j0 + jj] = Ps[j0 + p];
        Ps[j0 + p] = a;
      }
      __syncthreads();
      const int p = s_piv[jj];
      if (p != jj) {
        for (int c = tid; c < jb; c += 256) {
          const T a = Pn[jj + c * mr];
          Pn[jj + c * mr] = Pn[p + c * mr];
          Pn[p + c * mr] = a;
        }
      }
      __syncthreads();
      const T pv = Pn[jj + jj * mr];
      const bool ok = (pv != T(0)) && isfinite(pv);
      if (!ok) {
        if (tid == 0 && s_info == 0) s_info = j0 + jj + 1;
      } else {
        for (int r = jj + 1 + tid; r < mr; r += 256) Pn[r + jj * mr] /= pv;
      }
      __syncthreads();
      // rank-1 update of the rest of the panel
      const int rows = mr - jj - 1;
      const int cols = jb - jj - 1;
      for (int idx = tid; idx < rows * cols; idx += 256) {
        const int r = jj + 1 + idx % rows;
        const int c = jj + 1 + idx / rows;
        Pn[r + c * mr] -= Pn[r + jj * mr] * Pn[jj + c * mr];
      }
      __syncthreads();
    }

    // write the panel back
    for (int idx = tid; idx < mr * jb; idx += 256) {
      const int r = idx % mr, c = idx / mr;
      A[(int64_t)(j0 + c) * n + j0 + r] = Pn[r + c * mr];
    }
    // row interchanges on the columns outside the panel: compose the panel's
    // swaps into Loc (new row t takes old row Loc[t]) and move only the
    // touched rows
    for (int i = tid; i < mr; i += 256) Loc[i] = i;
    __syncthreads();
    if (tid == 0) {
      for (int jj = 0; jj < jb; ++jj) {
        const int p = s_piv[jj];
        const int a = Loc[jj];
        Loc[jj] = Loc[p];
        Loc[p] = a;
      }
      int cnt = 0;
      for (int jj = 0; jj < jb; ++jj) {
        const int cand[2] = {jj, s_piv[jj]};
        for (int q = 0; q < 2; ++q) {
          const int t = cand[q];
          if (Loc[t] == t) continue;
          bool dup = false;
          for (int u = 0; u < cnt; ++u) dup |= (s_tl[u] == t);
          if (!dup) s_tl[cnt++] = t;
        }
      }
      s_cnt = cnt;
    }
    __syncthreads();
    const int ncnt = s_cnt;
    const int nout = n - jb;
    if (ncnt > 0) {
      for (int q = tid; q < nout; q += 256) {
        const int c = (q < j0) ? q : q + jb;
        T* col = A + (int64_t)c * n + j0;
        T v[2 * NB];
#pragma unroll
        for (int u = 0; u < 2 * NB; ++u)
          if (u < ncnt) v[u] = col[Loc[s_tl[u]]];
#pragma unroll
        for (int u = 0; u < 2 * NB; ++u)
          if (u < ncnt) col[s_tl[u]] = v[u];
      }
    }
    __syncthreads();

    const int c0 = j0 + jb;
    const int m2 = n - c0;
    if (m2 > 0) {
      // U12 = L11^-1 A12, one thread per column
      for (int c = c0 + tid; c < n; c += 256) {
        T* col = A + (int64_t)c * n + j0;
        T u[NB];
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          if (jj < jb) {
            T v = col[jj];
#pragma unroll
            for (int t = 0; t < NB; ++t)
              if (t < jj) v -= Pn[jj + t * mr] * u[t];
            u[jj] = v;
          }
        }
#pragma unroll
        for (int jj = 0; jj < NB; ++jj)
          if (jj < jb) {
            col[jj] = u[jj];
            Us[jj * n + c] = u[jj];
          }
      }
      __syncthreads();
      // A22 -= L21 U12 with 4 x 4 register blocks
      const int nrb = (m2 + 3) / 4;
      const int nblk = nrb * nrb;
      for (int bidx = tid; bidx < nblk; bidx += 256) {
        const int r0 = c0 + (bidx % nrb) * 4;
        const int cc0 = c0 + (bidx / nrb) * 4;
        T acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = 0;
        for (int jj = 0; jj < jb; ++jj) {
          T a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = r0 + i;
            a[i] = (r < n) ? Pn[(r - j0) + jj * mr] : T(0);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int c = cc0 + j;
            b[j] = (c < n) ? Us[jj * n + c] : T(0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = cc0 + j;
          if (c >= n) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = r0 + i;
            if (r < n) A[(int64_t)c * n + r] -= acc[i][j];
          }
        }
      }
    }
    __syncthreads();
  }

  for (int i = tid; i < n; i += 256) pr.perm[i] = Ps[i];
  if (tid == 0) *pr.info = s_info;
}

template <typename T, int NB>
size_t getrf_smem(int nmax) {
  return (size_t)2 * nmax * NB * sizeof(T) + (size_t)2 * nmax * sizeof(int) + 16;
}

template <typename T, int NB>
hipError_t run_getrf(const LuProb* probs, int count, int nmax, hipStream_t s) {
  const size_t sm = getrf_smem<T, NB>(nmax);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrf<T, NB>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_getrf<T, NB>), dim3(count), dim3(256), sm, s, probs);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_getrf(const LuProb* probs, int count, int nmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  constexpr size_t kLds = 160 * 1024 - 1024;
  if (getrf_smem<T, 16>(nmax) <= kLds) return run_getrf<T, 16>(probs, count, nmax, s);
  if (getrf_smem<T, 8>(nmax) <= kLds) return run_getrf<T, 8>(probs, count, nmax, s);
  return run_getrf<T, 4>(probs, count, nmax, s);
}

template hipError_t launch_getrf<double>(const LuProb*, int, int, hipStream_t);
template hipError_t launch_getrf<float>(const LuProb*, int, int, hipStream_t);

}  // namespace invaskit
