// Batched LU with partial pivoting for square matrices of uneven order (the
// leaf LU of Algorithm 1 and the LU of the reduced systems of eq. (11)), one
// workgroup of NW waves per matrix (4, or 8 for the leaf blocks when the
// tuner finds it faster), every matrix of a launch in one grid.
//
// Matrices are row-major and rows never move: P A = L U is stored with
// logical row j of the packed L\U (unit-lower L below the diagonal, U on and
// above) in physical row perm[j], which is also the original row that the
// pivoting placed at position j.  Consumers read factor rows through perm,
// which costs nothing extra for row-wise operand loads and removes every
// row interchange from the factorization.  Right-looking blocked algorithm
// with panels of W columns (32 in FP32, 16 in FP64):
//   1. Panel.  The panel's rows are gathered into registers across the
//      workgroup (logical row j0 + r in thread r % NT, slot r / NT), each
//      carrying its logical position.  Per column: every wave finds its
//      candidate (the first row of largest magnitude: LAPACK getrf
//      semantics) and the owning lane publishes that row in LDS; one
//      barrier; every thread picks the winner of the NW, exchanges the two
//      logical positions, scales by the pivot's reciprocal and updates its
//      rows -- one barrier per column (the candidate rows are
//      double-buffered).
//   2. The panel goes back to the rows it came from, the permutation takes
//      the panel's logical positions, and inv(L11) is formed in LDS.
//   3. Panels come in pairs (superpanels of 2W columns): after panel a only
//      panel b's W columns are updated; after panel b the rest of the
//      trailing matrix is updated once with K = 2W, using the inverse of the
//      superpanel's unit-lower block.  Each update: for each chunk of 64
//      columns, U12 = inv(L11) A12 and A22 -= L21 U12 on the matrix cores
//      (16 x 16 tiles), L21 read as 16-byte row segments (load_row_sigma).
// info = j+1 for the first zero or non-finite pivot in column j (the column
// is left unscaled and the factorization continues, as LAPACK does).  KIND
// only separates the kernel names of the two uses (leaf blocks, reduced
// systems).
//
// PIV = false (leaf blocks lambda I + K_aa, symmetric positive definite for
// lambda > 0): no row exchanges.  The panel's W x W diagonal block is
// factored by one wave in registers, the rows below solve against it on the
// matrix cores, and the superpanel updates use the symmetry: only the rows
// at or below each column chunk are updated, and U12 = D L21^T comes from
// the final multipliers (D = the superpanel's pivots), which halves the
// trailing products.  The packed L\U written is the same as with pivoting
// (permutation = identity).  info flags the first pivot that is not
// positive and finite; the caller then factors again with pivoting.
#include <cmath>
#include <utility>

#include "device_util.hpp"
#include "internal.hpp"

namespace invaskit {
namespace {


// Pivot search keys.  For |a| >= 0 the IEEE bit pattern orders like an
// unsigned integer, so the largest magnitude is an integer max; key 0 marks
// "no candidate" (candidates carry bits + 1; a NaN counts as infinity and is
// flagged when it becomes the pivot).
__device__ __forceinline__ uint32_t abs_key(float v) {
  const float a = (v == v) ? fabsf(v) : INFINITY;
  return __builtin_bit_cast(uint32_t, a) + 1u;
}
__device__ __forceinline__ uint64_t abs_key(double v) {
  const double a = (v == v) ? fabs(v) : (double)INFINITY;
  return __builtin_bit_cast(uint64_t, a) + 1ull;
}
template <typename T>
using key_t = decltype(abs_key(T(0)));

// DPP lane exchanges inside each 16-lane row: xor 1, xor 2 (quad_perm),
// half-row mirror, row mirror -- a butterfly that leaves the row's maximum
// (minimum) in every lane.  Rows are then combined through readlane.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp(uint64_t x) {
  const uint32_t lo = dpp<CTRL>((uint32_t)x), hi = dpp<CTRL>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rlane(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ uint64_t rlane(uint64_t x, int l) {
  return ((uint64_t)rlane((uint32_t)(x >> 32), l) << 32) | rlane((uint32_t)x, l);
}
constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
template <typename U>
__device__ __forceinline__ U wave_max(U k) {
  U o;
  o = dpp<kXor1>(k); k = o > k ? o : k;
  o = dpp<kXor2>(k); k = o > k ? o : k;
  o = dpp<kHalfMirror>(k); k = o > k ? o : k;
  o = dpp<kMirror>(k); k = o > k ? o : k;
  const U a = rlane(k, 0), b = rlane(k, 16), c = rlane(k, 32), d = rlane(k, 48);
  const U ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}
__device__ __forceinline__ uint32_t wave_min(uint32_t k) {
  uint32_t o;
  o = dpp<kXor1>(k); k = o < k ? o : k;
  o = dpp<kXor2>(k); k = o < k ? o : k;
  o = dpp<kHalfMirror>(k); k = o < k ? o : k;
  o = dpp<kMirror>(k); k = o < k ? o : k;
  const uint32_t a = rlane(k, 0), b = rlane(k, 16), c = rlane(k, 32), d = rlane(k, 48);
  const uint32_t ab = a < b ? a : b, cd = c < d ? c : d;
  return ab < cd ? ab : cd;
}

// 1 / p: FP32 by the hardware reciprocal and one Newton step (LAPACK also
// scales by the reciprocal), plain division below FLT_MIN and in FP64
__device__ __forceinline__ float recip(float p) {
  if (fabsf(p) < 1.17549435e-38f) return 1.0f / p;
  const float r = __builtin_amdgcn_rcpf(p);
  return fmaf(r, fmaf(-p, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double p) { return 1.0 / p; }

constexpr int CH = 64;  // column chunk of the U12 / trailing update

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename T, int W, int RPS, int KIND, int NW, bool PIV>
__global__ __launch_bounds__(64 * NW) void k_getrf(const LuProb* __restrict__ probs) {
  using V4 = typename Vec4<T>::type;
  constexpr int W2 = 2 * W;
  constexpr int NT = 64 * NW;  // threads
  static_assert(W % NW == 0, "inv(L11) gives each wave W / NW columns");
  const LuProb pr = probs[blockIdx.x];
  const gptr<T> A = glb(static_cast<T*>(pr.a));
  const int n = pr.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar branches
  const int lr = lane & 15, lg = lane >> 4;

  extern __shared__ __align__(16) unsigned char smem[];
  int* Ps = reinterpret_cast<int*>(smem);  // logical row -> physical row, n entries
  __shared__ __align__(16) T s_row[2][NW][W];  // each wave's candidate pivot row
  __shared__ __align__(16) key_t<T> s_bk[2][NW];
  __shared__ __align__(16) uint32_t s_bl[2][NW];
  __shared__ T L11[W][W + 1];              // a panel's unit-lower block, then L21_ab
  __shared__ T Lsup[W2][W2 + 1];           // inverse of the 2W superpanel's unit-lower block
  __shared__ T Uc[W2][CH];                 // U12 chunk
  __shared__ T s_dinv[W];                  // without pivoting: 1 / U11's diagonal
  __shared__ T Ui[W][W + 1];               // without pivoting: inv(U11)
  __shared__ T s_dsup[W2];                 // without pivoting: the superpanel's pivots
  __shared__ int s_info;

  for (int i = tid; i < n; i += NT) Ps[i] = i;
  if (tid == 0) s_info = 0;
  __syncthreads();

  // ---- inv(L11) (unit lower, from L11) into Lsup[off .. off+W)^2: wave w
  // solves identity columns w*W/NW .. +W/NW, lane = row, the solved row
  // value broadcast across lanes
  auto l11_inverse = [&](int jb, int off) {
    {
      constexpr int CQ = W / NW;
      T x[CQ];
#pragma unroll
      for (int q = 0; q < CQ; ++q) x[q] = (lane == wave * CQ + q) ? T(1) : T(0);
      for (int j = 0; j < jb - 1; ++j) {
        const T l = (lane > j && lane < jb) ? L11[lane][j] : T(0);
#pragma unroll
        for (int q = 0; q < CQ; ++q) x[q] -= l * lane_bcast(x[q], j);
      }
      if (lane < W) {
#pragma unroll
        for (int q = 0; q < CQ; ++q)
          Lsup[off + lane][off + wave * CQ + q] = (lane < jb) ? x[q] : T(0);
      }
    }
    __syncthreads();
  };

  // ---- factor the W columns at j0 (rows >= j0), write them back in place,
  // give the panel's rows their logical positions, and put inv(L11) in
  // Lsup[off .. off+W)[off .. off+W).  Returns the panel width.
  auto panel = [&](int j0, int off) -> int {
    const int jb = min(W, n - j0);
    const int mr = n - j0;
    T P[RPS][W];
    int lpos[RPS], ph[RPS];
#pragma unroll
    for (int t = 0; t < RPS; ++t) {
      const int r = tid + NT * t;
      lpos[t] = (r < mr) ? r : -1;
      ph[t] = (r < mr) ? Ps[j0 + r] : 0;
#pragma unroll
      for (int c = 0; c < W; ++c)
        P[t][c] = (r < mr && c < jb) ? A[(int64_t)ph[t] * n + j0 + c] : T(0);
    }
    int info = 0;
    static_for<W>([&](auto JJ) {
      constexpr int jj = decltype(JJ)::value;
      if (jj < jb) {
      const int buf = jj & 1;
      // this thread's best candidate: largest |a|, then the smaller row
      key_t<T> bk = 0;
      uint32_t bl = 0xffffffffu;
#pragma unroll
      for (int t = 0; t < RPS; ++t) {
        if (lpos[t] >= jj) {
          const key_t<T> k = abs_key(P[t][jj]);
          if (k > bk || (k == bk && (uint32_t)lpos[t] < bl)) {
            bk = k;
            bl = (uint32_t)lpos[t];
          }
        }
      }
      const key_t<T> wk = wave_max(bk);
      const uint32_t wl = wave_min(bk == wk ? bl : 0xffffffffu);
      // the owning lane publishes the wave's candidate row (predicated
      // stores per slot: a select over slots would index P in memory)
#pragma unroll
      for (int t = 0; t < RPS; ++t) {
        if ((uint32_t)lpos[t] == wl) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_row[buf][wave][c] = P[t][c];
        }
      }
      if (lane == 0) {
        s_bk[buf][wave] = wk;
        s_bl[buf][wave] = wl;
      }
      __syncthreads();
      // every wave's candidate in one round of LDS reads, the winner (largest
      // key, then the smaller logical row) by selects, then its row in one
      // more round: two dependent LDS latencies per column
      key_t<T> kv[NW];
      uint32_t lv[NW];
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        kv[ww] = s_bk[buf][ww];
        lv[ww] = s_bl[buf][ww];
      }
      int w = 0;
      key_t<T> kbest = kv[0];
      uint32_t plu = lv[0];
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) {
        const bool better = kv[ww] > kbest || (kv[ww] == kbest && lv[ww] < plu);
        kbest = better ? kv[ww] : kbest;
        plu = better ? lv[ww] : plu;
        w = better ? ww : w;
      }
      const int pl = (int)plu;
      T prow[W];
#pragma unroll
      for (int c = 0; c < W; ++c) prow[c] = (c >= jj) ? s_row[buf][w][c] : T(0);
      const T pv = prow[jj];
      const bool ok = (pv != T(0)) && isfinite(pv);
      if (!ok && info == 0) info = j0 + jj + 1;
#pragma unroll
      for (int t = 0; t < RPS; ++t) {
        if (lpos[t] == pl)
          lpos[t] = jj;
        else if (lpos[t] == jj)
          lpos[t] = pl;
      }
      if (ok) {
        const T inv = recip(pv);
#pragma unroll
        for (int t = 0; t < RPS; ++t) {
          if (lpos[t] > jj) {
            const T l = P[t][jj] * inv;
            P[t][jj] = l;
#pragma unroll
            for (int c = jj + 1; c < W; ++c) P[t][c] -= l * prow[c];
          }
        }
      }
      }
    });
    // write back in place, new logical order (every thread read its Ps
    // entries before the panel's first barrier)
    if (tid == 0 && info != 0 && s_info == 0) s_info = info;
#pragma unroll
    for (int t = 0; t < RPS; ++t) {
      const int lp = lpos[t];
      if (lp >= 0) {
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < jb) A[(int64_t)ph[t] * n + j0 + c] = P[t][c];
        if (lp < W) {
#pragma unroll
          for (int c = 0; c < W; ++c) L11[lp][c] = P[t][c];
        }
        Ps[j0 + lp] = ph[t];
      }
    }
    __syncthreads();
    l11_inverse(jb, off);
    return jb;
  };

  // ---- the same panel without pivoting, for symmetric positive definite
  // blocks (the leaf blocks lambda I + K_aa with lambda > 0), where LU with
  // no row exchanges is backward stable and the pivots are the positive
  // diagonal of the LDL^T factorization.  Rows keep their order (the
  // permutation stays the identity).  Wave 0 factors the W x W diagonal
  // block in registers (lane i = row i, the pivot row broadcast by
  // readlane, no barrier); the waves form inv(U11) beside inv(L11); the rows
  // below become L21 = A21 inv(U11) on the matrix cores, 16 rows per tile.
  // No step waits on a barrier per column.  A pivot that is not positive
  // and finite sets info (the caller then factors again with pivoting).
  auto panel_np = [&](int j0, int off) -> int {
    const int jb = min(W, n - j0);
    if (wave == 0) {
      T P0[W];
      const gptr<T> rowp = A + (int64_t)(j0 + (lane < jb ? lane : 0)) * n + j0;
#pragma unroll
      for (int c = 0; c < W; ++c) P0[c] = (lane < jb && c < jb) ? rowp[c] : T(0);
      int info = 0;
      static_for<W>([&](auto JJ) {
        constexpr int jj = decltype(JJ)::value;
        if (jj < jb) {
          T prow[W];
#pragma unroll
          for (int c = 0; c < W; ++c) prow[c] = (c >= jj) ? lane_bcast(P0[c], jj) : T(0);
          const T pv = prow[jj];
          const bool ok = pv > T(0) && isfinite(pv);
          if (!ok && info == 0) info = j0 + jj + 1;
          if (lane > jj && lane < jb) {
            const T l = P0[jj] * recip(pv);
            P0[jj] = l;
#pragma unroll
            for (int c = jj + 1; c < W; ++c) P0[c] -= l * prow[c];
          }
        }
      });
      if (lane < jb) {
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < jb) rowp[c] = P0[c];
      }
      if (lane < W) {
#pragma unroll
        for (int c = 0; c < W; ++c) L11[lane][c] = (lane < jb) ? P0[c] : T(0);
        // each lane reads back its own diagonal entry (same thread: ordered)
        s_dinv[lane] = (lane < jb) ? recip(L11[lane][lane]) : T(0);
        s_dsup[off + lane] = (lane < jb) ? L11[lane][lane] : T(0);
      }
      if (lane == 0 && info != 0 && s_info == 0) s_info = info;
    }
    __syncthreads();
    // inv(U11) into Ui: wave w solves identity columns w*W/NW .. +W/NW by
    // back substitution, lane = row; once row j is divided by u_jj it is
    // final and is broadcast to the rows above
    {
      constexpr int CQ = W / NW;
      T x[CQ];
#pragma unroll
      for (int q = 0; q < CQ; ++q) x[q] = (lane == wave * CQ + q) ? T(1) : T(0);
      for (int j = jb - 1; j >= 0; --j) {
        const T dj = s_dinv[j];
        const T u = (lane < j) ? L11[lane < W ? lane : 0][j] : T(0);
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
          if (lane == j) x[q] *= dj;
          x[q] -= u * lane_bcast(x[q], j);
        }
      }
      if (lane < W) {
#pragma unroll
        for (int q = 0; q < CQ; ++q) Ui[lane][wave * CQ + q] = (lane < jb) ? x[q] : T(0);
      }
    }
    l11_inverse(jb, off);  // ends with a barrier: Ui and Lsup are complete
    // L21 = A21 inv(U11).  Rows below exist only when the panel is W wide,
    // so a row's W panel entries are always inside the row.
    // Each wave takes its tiles four at a time, all four loads in flight
    // before the first product.
    constexpr int NBT = 4;
    const int r0 = j0 + jb;
    const int ntr = (n - r0 + 15) / 16;
    for (int it0 = wave; it0 < ntr; it0 += NBT * NW) {
      T a[NBT][W / 4];
#pragma unroll
      for (int q = 0; q < NBT; ++q) {
        const int row = r0 + 16 * (it0 + q * NW) + lr;
        load_row_sigma_full(A + (int64_t)(row < n ? row : r0 - 1) * n + j0, row < n ? W : 0, lg,
                            a[q]);
      }
#pragma unroll
      for (int q = 0; q < NBT; ++q) {
        const int t0 = r0 + 16 * (it0 + q * NW);
        if (t0 < n) {
#pragma unroll
          for (int ct = 0; ct < W / 16; ++ct) {
            V4 acc = V4{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < W / 4; ++kk)
              acc = mfma16(a[q][kk], Ui[sigma_k<T>(kk, lg)][16 * ct + lr], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int rr = t0 + acc_row(T(0), lg, v);
              if (rr < n) A[(int64_t)rr * n + j0 + 16 * ct + lr] = acc[v];
            }
          }
        }
      }
    }
    __syncthreads();
    return jb;
  };

  // ---- trailing update of the rows below logical row r0 + KW, columns
  // [cs, ce), by the KW rows at r0: U12 = Lsup[0..KW)^2 A12 per 64-column
  // chunk (written back as rows r0+1 .. r0+KW-1 of U), then A22 -= L21 U12,
  // both on the matrix cores, L21 read as 16-byte row segments.
  auto update = [&](auto KWc, int r0, int cs, int ce) {
    constexpr int KW = decltype(KWc)::value;
    constexpr int KG = KW / 4;
    // Without pivoting the trailing matrix stays symmetric: a superpanel
    // updates only the rows at or below each column chunk (half the
    // products), and its U12 rows, whose entries right of the chunk's
    // diagonal are then stale, are formed from the final L21 instead:
    // U12 = D L21^T (D = the superpanel's pivots).
    constexpr bool SYM = !PIV && KW == W2;
    const int c0 = r0 + KW;
    for (int cb = cs; cb < ce; cb += CH) {
      const int rs = SYM ? cb : c0;  // first row of the chunk's update
      const int ntr = (n - rs + 15) / 16;
      if constexpr (SYM) {
        for (int idx = tid; idx < KW * CH; idx += NT) {
          const int cl = idx / KW, k = idx % KW;  // consecutive threads: one L row
          const int cc = cb + cl;
          Uc[k][cl] = (cc < ce) ? s_dsup[k] * A[(int64_t)cc * n + r0 + k] : T(0);
        }
      }
      // wave w takes the chunk's 16-column blocks w, w + NW, ...: it loads
      // a block's KW rows of A12 once and applies every row block of Lsup
      if constexpr (!SYM) for (int ct = wave; ct < CH / 16; ct += NW) {
        const int cc = cb + 16 * ct + lr;
        T b[KG];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
          b[kk] = (cc < ce) ? A[(int64_t)Ps[r0 + 4 * kk + lg] * n + cc] : T(0);
#pragma unroll
        for (int rt = 0; rt < KW / 16; ++rt) {
          V4 acc = V4{0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < KG; ++kk) acc = mfma16(Lsup[16 * rt + lr][4 * kk + lg], b[kk], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) Uc[16 * rt + acc_row(T(0), lg, v)][16 * ct + lr] = acc[v];
        }
      }
      __syncthreads();
      // write U12 back (logical rows r0+1 .. r0+KW-1; row r0 is unchanged,
      // except in the symmetric form, where it is rewritten too)
      for (int idx = tid; idx < KW * CH; idx += NT) {
        const int i = idx / CH, cl = idx % CH;
        const int cc = cb + cl;
        if ((SYM || i >= 1) && cc < ce) A[(int64_t)Ps[r0 + i] * n + cc] = Uc[i][cl];
      }
      // two row tiles per iteration (it and it + NW), and in FP32 the next
      // iteration's two tiles are loaded while this one computes (FP64
      // has no registers to spare).  r0 + KW <= n here, so a row's segment
      // lies inside the row; rows past the last read row Ps[0] instead
      // (their products are never stored), so the loads are unmasked and
      // wait only where the products use them, and the loop has no
      // divergent path.
      constexpr int CTB = (CH / 16) * W / KW;  // 16-column blocks per pass
      constexpr bool PREF = sizeof(T) == 4;
      auto row_tile = [&](int it, T (&a)[KG], int (&pr4)[4]) {
        const int t0 = rs + 16 * it;
        const int row = t0 + lr;
        load_row_sigma_raw((gptr<const T>)(A + (int64_t)Ps[row < n ? row : 0] * n + r0), lg, a);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = t0 + acc_row(T(0), lg, v);
          pr4[v] = (rr < n) ? Ps[rr] : -1;
        }
      };
      T a0[KG], a1[KG];
      int p0[4], p1[4];
      if (wave < ntr) {
        row_tile(wave, a0, p0);
        row_tile(wave + NW, a1, p1);
      }
      for (int it = wave; it < ntr; it += 2 * NW) {
        const bool more = it + 2 * NW < ntr;
        T b0[PREF ? KG : 1], b1[PREF ? KG : 1];
        int q0[4], q1[4];
        if constexpr (PREF) {
          if (more) {
            row_tile(it + 2 * NW, b0, q0);
            row_tile(it + 3 * NW, b1, q1);
          }
        }
        // the chunk's 16-column blocks in passes of CTB, so that K = 2W keeps
        // about as many operands live as K = W
#pragma unroll
        for (int c1 = 0; c1 < CH / 16; c1 += CTB) {
          V4 cur0[CTB], cur1[CTB];
#pragma unroll
          for (int q = 0; q < CTB; ++q) {
            const int cc = cb + 16 * (c1 + q) + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              cur0[q][v] = (p0[v] >= 0 && cc < ce) ? A[(int64_t)p0[v] * n + cc] : T(0);
              cur1[q][v] = (p1[v] >= 0 && cc < ce) ? A[(int64_t)p1[v] * n + cc] : T(0);
            }
          }
#pragma unroll
          for (int q = 0; q < CTB; ++q) {
            V4 acc0 = V4{0, 0, 0, 0}, acc1 = V4{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
              const T u = Uc[sigma_k<T>(kk, lg)][16 * (c1 + q) + lr];
              acc0 = mfma16(a0[kk], u, acc0);
              acc1 = mfma16(a1[kk], u, acc1);
            }
            const int cc = cb + 16 * (c1 + q) + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (p0[v] >= 0 && cc < ce) A[(int64_t)p0[v] * n + cc] = cur0[q][v] - acc0[v];
              if (p1[v] >= 0 && cc < ce) A[(int64_t)p1[v] * n + cc] = cur1[q][v] - acc1[v];
            }
          }
        }
        if (more) {
          if constexpr (PREF) {
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
              a0[kk] = b0[kk];
              a1[kk] = b1[kk];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              p0[v] = q0[v];
              p1[v] = q1[v];
            }
          } else {
            row_tile(it + 2 * NW, a0, p0);
            row_tile(it + 3 * NW, a1, p1);
          }
        }
      }
      __syncthreads();
    }
  };

  // Superpanels of 2W columns: panel a, the update of panel b's columns by
  // panel a, panel b, then one pass over the rest of the trailing matrix
  // with K = 2W -- half the passes of a W-wide schedule, with the panels
  // still W wide in registers.  Rows never move, so panel a's multipliers
  // stay valid under panel b's pivoting.  One panel per iteration (the
  // panel code is inlined once).
  for (int j0 = 0; j0 < n; j0 += W) {
    const bool second = ((j0 / W) & 1) != 0;  // panel b of its superpanel
    if constexpr (PIV)
      panel(j0, second ? W : 0);
    else
      panel_np(j0, second ? W : 0);
    if (j0 + W >= n) break;  // nothing to the right
    if (!second) {
      update(std::integral_constant<int, W>{}, j0, j0 + W, min(n, j0 + W2));
      continue;
    }
    // Both panels of the superpanel at J0 are full.  Its unit-lower block
    // is [[L_a, 0], [L_ab, L_b]]; the inverse has the lower-left block
    // X = -inv(L_b) L_ab inv(L_a), with L_ab = panel b's rows in panel a's
    // columns.
    const int J0 = j0 - W;
    if constexpr (!PIV) {
      // the symmetric update forms U12 from L21 and needs no inverse
      update(std::integral_constant<int, W2>{}, J0, J0 + W2, n);
      continue;
    }
    for (int idx = tid; idx < W * W; idx += NT) {
      const int i = idx / W, c = idx % W;
      L11[i][c] = A[(int64_t)Ps[J0 + W + i] * n + J0 + c];
      Lsup[i][W + c] = T(0);
    }
    __syncthreads();
    for (int it = wave; it < (W / 16) * (W / 16); it += NW) {  // Uc = L_ab inv(L_a)
      const int rt = it % (W / 16), ct = it / (W / 16);
      V4 acc = V4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < W / 4; ++kk)
        acc = mfma16(L11[16 * rt + lr][4 * kk + lg], Lsup[4 * kk + lg][16 * ct + lr], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) Uc[16 * rt + acc_row(T(0), lg, v)][16 * ct + lr] = acc[v];
    }
    __syncthreads();
    for (int it = wave; it < (W / 16) * (W / 16); it += NW) {  // X = -inv(L_b) Uc
      const int rt = it % (W / 16), ct = it / (W / 16);
      V4 acc = V4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < W / 4; ++kk)
        acc = mfma16(Lsup[W + 16 * rt + lr][W + 4 * kk + lg], Uc[4 * kk + lg][16 * ct + lr], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) Lsup[W + 16 * rt + acc_row(T(0), lg, v)][16 * ct + lr] = -acc[v];
    }
    __syncthreads();
    update(std::integral_constant<int, W2>{}, J0, J0 + W2, n);
  }

  for (int i = tid; i < n; i += NT) glb(pr.perm)[i] = Ps[i];
  if (tid == 0) *glb(pr.info) = s_info;
}

// One wave per matrix, for small orders (n <= 64 RPS; panels of 32 columns
// in FP32, 16 in FP64): the same blocked
// algorithm and storage as k_getrf, but with no workgroup barriers -- the
// pivot search is a wave reduction, the pivot row is broadcast by readlane
// from the owning lane, and the panel inverse, U12 and the trailing update
// are computed by the one wave.  This shortens the per-column chain, which
// is what bounds the small reduced systems near the root.
template <typename T, int W, int RPS, int KIND>
__global__ __launch_bounds__(64) void k_getrf_w(const LuProb* __restrict__ probs) {
  using V4 = typename Vec4<T>::type;
  const LuProb pr = probs[blockIdx.x];
  const gptr<T> A = glb(static_cast<T*>(pr.a));
  const int n = pr.n;
  const int lane = threadIdx.x;
  const int lr = lane & 15, lg = lane >> 4;

  extern __shared__ __align__(16) unsigned char smem[];
  int* Ps = reinterpret_cast<int*>(smem);  // logical row -> physical row, n entries
  __shared__ T L11[W][W + 1];
  __shared__ T Li[W][W + 1];
  __shared__ T Uc[W][CH];

  for (int i = lane; i < n; i += 64) Ps[i] = i;
  int info = 0;

  for (int j0 = 0; j0 < n; j0 += W) {
    const int jb = min(W, n - j0);
    const int mr = n - j0;
    T P[RPS][W];
    int lpos[RPS], ph[RPS];
#pragma unroll
    for (int t = 0; t < RPS; ++t) {
      const int r = lane + 64 * t;
      lpos[t] = (r < mr) ? r : -1;
      ph[t] = (r < mr) ? Ps[j0 + r] : 0;
#pragma unroll
      for (int c = 0; c < W; ++c)
        P[t][c] = (r < mr && c < jb) ? A[(int64_t)ph[t] * n + j0 + c] : T(0);
    }
    static_for<W>([&](auto JJ) {
      constexpr int jj = decltype(JJ)::value;
      if (jj < jb) {
        key_t<T> bk = 0;
        uint32_t bl = 0xffffffffu;
#pragma unroll
        for (int t = 0; t < RPS; ++t) {
          if (lpos[t] >= jj) {
            const key_t<T> k = abs_key(P[t][jj]);
            if (k > bk || (k == bk && (uint32_t)lpos[t] < bl)) {
              bk = k;
              bl = (uint32_t)lpos[t];
            }
          }
        }
        const key_t<T> wk = wave_max(bk);
        const uint32_t pl = wave_min(bk == wk ? bl : 0xffffffffu);
        // the owner: (slot, lane) of logical row pl, uniform after the reduction
        uint32_t code = 0xffffffffu;
#pragma unroll
        for (int t = 0; t < RPS; ++t)
          if ((uint32_t)lpos[t] == pl) code = ((uint32_t)t << 6) | (uint32_t)lane;
        code = wave_min(code);
        const int olane = (int)(code & 63u), oslot = (int)(code >> 6);
        T prow[W];
        static_for<RPS>([&](auto TT) {
          constexpr int t = decltype(TT)::value;
          if (oslot == t) {
#pragma unroll
            for (int c = 0; c < W; ++c) prow[c] = lane_bcast(P[t][c], olane);
          }
        });
        const T pv = prow[jj];
        const bool ok = (pv != T(0)) && isfinite(pv);
        if (!ok && info == 0) info = j0 + jj + 1;
#pragma unroll
        for (int t = 0; t < RPS; ++t) {
          if (lpos[t] == (int)pl)
            lpos[t] = jj;
          else if (lpos[t] == jj)
            lpos[t] = (int)pl;
        }
        if (ok) {
          const T inv = recip(pv);
#pragma unroll
          for (int t = 0; t < RPS; ++t) {
            if (lpos[t] > jj) {
              const T l = P[t][jj] * inv;
              P[t][jj] = l;
#pragma unroll
              for (int c = jj + 1; c < W; ++c) P[t][c] -= l * prow[c];
            }
          }
        }
      }
    });
    // write back in place, new logical order, inverse of L11 (one wave: the
    // LDS accesses of a wave complete in order, so no barrier is needed)
#pragma unroll
    for (int t = 0; t < RPS; ++t) {
      const int lp = lpos[t];
      if (lp >= 0) {
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < jb) A[(int64_t)ph[t] * n + j0 + c] = P[t][c];
        if (lp < W) {
#pragma unroll
          for (int c = 0; c < W; ++c) L11[lp][c] = P[t][c];
        }
        Ps[j0 + lp] = ph[t];
      }
    }
    __builtin_amdgcn_wave_barrier();
    {
      T x[W];
#pragma unroll
      for (int q = 0; q < W; ++q) x[q] = (lane == q) ? T(1) : T(0);
      for (int j = 0; j < jb - 1; ++j) {
        const T l = (lane > j && lane < jb) ? L11[lane][j] : T(0);
#pragma unroll
        for (int q = 0; q < W; ++q) x[q] -= l * lane_bcast(x[q], j);
      }
      if (lane < W) {
#pragma unroll
        for (int q = 0; q < W; ++q) Li[lane][q] = (lane < jb) ? x[q] : T(0);
      }
    }
    int uph[W / 4];
#pragma unroll
    for (int kk = 0; kk < W / 4; ++kk) {
      const int k = 4 * kk + lg;
      uph[kk] = (k < jb) ? Ps[j0 + k] : 0;
    }
    __builtin_amdgcn_wave_barrier();
    const int c0 = j0 + jb;
    for (int cb = c0; cb < n; cb += CH) {
      // each 16-column block of A12 is loaded once for both row blocks
      for (int ct = 0; ct < CH / 16; ++ct) {
        const int cc = cb + 16 * ct + lr;
        T b[W / 4];
#pragma unroll
        for (int kk = 0; kk < W / 4; ++kk) {
          const int k = 4 * kk + lg;
          b[kk] = (cc < n && k < jb) ? A[(int64_t)uph[kk] * n + cc] : T(0);
        }
#pragma unroll
        for (int rt = 0; rt < W / 16; ++rt) {
          V4 acc = V4{0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < W / 4; ++kk) acc = mfma16(Li[16 * rt + lr][4 * kk + lg], b[kk], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) Uc[16 * rt + acc_row(T(0), lg, v)][16 * ct + lr] = acc[v];
        }
      }
      __builtin_amdgcn_wave_barrier();
      for (int idx = lane; idx < W * CH; idx += 64) {
        const int i = idx / CH, cl = idx % CH;
        const int cc = cb + cl;
        if (i >= 1 && i < jb && cc < n) A[(int64_t)Ps[j0 + i] * n + cc] = Uc[i][cl];
      }
      const int ntr = (n - c0 + 15) / 16;
      for (int it = 0; it < ntr; ++it) {
        const int t0 = c0 + 16 * it;
        const int row = t0 + lr;
        constexpr int KG = W / 4;
        T a[KG];
        load_row_sigma_full(A + (int64_t)(row < n ? Ps[row] : 0) * n + j0, row < n ? W : 0, lg, a);
        int pr4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = t0 + acc_row(T(0), lg, v);
          pr4[v] = (rr < n) ? Ps[rr] : -1;
        }
        V4 cur[CH / 16];
#pragma unroll
        for (int ct = 0; ct < CH / 16; ++ct) {
          const int cc = cb + 16 * ct + lr;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            cur[ct][v] = (pr4[v] >= 0 && cc < n) ? A[(int64_t)pr4[v] * n + cc] : T(0);
        }
#pragma unroll
        for (int ct = 0; ct < CH / 16; ++ct) {
          V4 acc = V4{0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < KG; ++kk)
            acc = mfma16(a[kk], Uc[sigma_k<T>(kk, lg)][16 * ct + lr], acc);
          const int cc = cb + 16 * ct + lr;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (pr4[v] >= 0 && cc < n) A[(int64_t)pr4[v] * n + cc] = cur[ct][v] - acc[v];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  for (int i = lane; i < n; i += 64) glb(pr.perm)[i] = Ps[i];
  if (lane == 0) *glb(pr.info) = info;
}

template <typename T, int W, int RPS, int KIND>
hipError_t run_getrf_w(const LuProb* probs, int count, int nmax, hipStream_t s) {
  const size_t sm = (size_t)nmax * sizeof(int);
  hipLaunchKernelGGL((k_getrf_w<T, W, RPS, KIND>), dim3(count), dim3(64), sm, s, probs);
  return hipGetLastError();
}

template <typename T, int W, int RPS, int KIND, int NW, bool PIV>
hipError_t run_getrf(const LuProb* probs, int count, int nmax, hipStream_t s) {
  const size_t sm = (size_t)nmax * sizeof(int);
  hipLaunchKernelGGL((k_getrf<T, W, RPS, KIND, NW, PIV>), dim3(count), dim3(64 * NW), sm, s,
                     probs);
  return hipGetLastError();
}

// RPS rows of the panel per thread: orders up to 64 NW RPS
template <typename T, int W, int KIND, int NW, bool PIV>
hipError_t run_block(const LuProb* probs, int count, int nmax, hipStream_t s) {
  constexpr int NT = 64 * NW;
  if (nmax <= NT) return run_getrf<T, W, 1, KIND, NW, PIV>(probs, count, nmax, s);
  if (nmax <= 2 * NT) return run_getrf<T, W, 2, KIND, NW, PIV>(probs, count, nmax, s);
  if constexpr (NW == 4) {
    if (nmax <= 4 * NT) return run_getrf<T, W, 4, KIND, NW, PIV>(probs, count, nmax, s);
  }
  return hipErrorInvalidValue;
}

// panel: 0 = the default width (32 in FP32, 16 in FP64), else 16 or 32;
// waves: 0 or 4 = four waves per matrix, 8 = eight (leaf blocks only; the
// reduced systems always take the defaults; FP64 has no panel 32 at eight
// waves).  Orders up to kOneWaveMax may take the one-wave kernel (panel 32
// in FP32, 16 in FP64): by default in FP32, whose short per-column chain is
// what bounds the small reduced systems near the root; FP64's longer chain
// (64-bit keys and reciprocal) is spread over four waves unless `form` asks
// for the one-wave kernel.
template <typename T, int KIND, bool PIV>
hipError_t pick_block(const LuProb* probs, int count, int nmax, int panel, int waves,
                      hipStream_t s) {
  constexpr int W = sizeof(T) == 8 ? 16 : 32;
  constexpr int WA = W == 16 ? 32 : 16;  // the other panel width
  const bool alt = panel != 0 && panel != W;
  if (alt && panel != WA) return hipErrorInvalidValue;
  if (waves != 0 && waves != 4 && waves != 8) return hipErrorInvalidValue;
  if (!alt && waves != 8) return run_block<T, W, KIND, 4, PIV>(probs, count, nmax, s);
  if constexpr (KIND == 0) {
    if (!alt) return run_block<T, W, KIND, 8, PIV>(probs, count, nmax, s);
    if (waves != 8) return run_block<T, WA, KIND, 4, PIV>(probs, count, nmax, s);
    // FP64 with panel 32 at eight waves would spill registers: not built
    if constexpr (sizeof(T) == 4) return run_block<T, WA, KIND, 8, PIV>(probs, count, nmax, s);
  }
  return hipErrorInvalidValue;
}

// nopiv (leaf blocks only): the block kernel without row exchanges; the
// one-wave kernel always pivots
template <typename T, int KIND>
hipError_t pick(const LuProb* probs, int count, int nmax, int panel, int waves, int form,
                bool nopiv, hipStream_t s) {
  constexpr int W = sizeof(T) == 8 ? 16 : 32;
  const bool one = nmax <= kOneWaveMax &&
                   (form == kLuFormOneWave || (form == kLuFormAuto && sizeof(T) == 4));
  if (one) {
    if (nmax <= 64) return run_getrf_w<T, W, 1, KIND>(probs, count, nmax, s);
    if (nmax <= 128) return run_getrf_w<T, W, 2, KIND>(probs, count, nmax, s);
    return run_getrf_w<T, W, 3, KIND>(probs, count, nmax, s);
  }
  if constexpr (KIND == 0) {
    if (nopiv) return pick_block<T, KIND, false>(probs, count, nmax, panel, waves, s);
  }
  return pick_block<T, KIND, true>(probs, count, nmax, panel, waves, s);
}

}  // namespace

int getrf_default_panel(bool t64) { return t64 ? 16 : 32; }

template <typename T>
hipError_t launch_getrf(const LuProb* probs, int count, int nmax, int kind, int panel, int waves,
                        hipStream_t s, int form, bool nopiv) {
  if (count <= 0) return hipSuccess;
  if (form < kLuFormAuto || form > kLuFormBlock) return hipErrorInvalidValue;
  return kind == 0 ? pick<T, 0>(probs, count, nmax, panel, waves, form, nopiv, s)
                   : pick<T, 1>(probs, count, nmax, panel, waves, form, false, s);
}

template hipError_t launch_getrf<double>(const LuProb*, int, int, int, int, int, hipStream_t, int,
                                         bool);
template hipError_t launch_getrf<float>(const LuProb*, int, int, int, int, int, hipStream_t, int,
                                        bool);

}  // namespace invaskit
