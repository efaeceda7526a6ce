// Gaussian kernel evaluation (eq. (1)), K(x,y) = exp(-|x-y|^2/(2h^2)).
//
// k_eval writes blocks of K: the leaf blocks lambda*I + K_{aa} of
// Algorithm 1 and the skeleton blocks K_{c, sibling~} of eq.
// (7), straight into the factor storage.  A workgroup computes
// a 64 x 64 tile: the 64 row points and 64 column points are staged through
// LDS in chunks of 8 coordinates and every thread accumulates a 4 x 4 block
// of squared distances by direct differences in FP64 (no |x|^2+|y|^2-2x.y
// cancellation), then applies exp and stores in the factor precision.
//
// k_mv_eval is the fused FP64 evaluate step of the hierarchical product
// (Section II-B, Evaluate): one thread per target point keeps its
// coordinates in registers (d <= 64); source points and their weights are
// staged through LDS 64 at a time and K(x_i, x_j) is consumed immediately,
// so the kernel matrix is never stored.  Its exponents are formed in the
// shifted Gram form and its exp is a table-driven one (exp_nonpos): about
// 24 vector operations per pair instead of 38.
//
// Above d = 64 the squared distances are a dense contraction over the
// coordinates, so both kernels switch to the Gram form on the matrix cores
// (k_eval_gram, k_mv_eval_gram): |x - y|^2 = |x'|^2 + |y'|^2 - 2 x'.y' with
// x' = x - z, y' = y - z for a reference point z of the tile (its first row
// point; the distance does not depend on z, and the shift keeps the norms,
// and so the cancellation, at the scale of the distances).  The products run
// in FP64 on the matrix cores whatever the output precision: an FP32 Gram
// over hundreds of coordinates would carry distance errors about sqrt(d)
// times FP32 rounding, well above the FP32 rounding of the stored kernel
// value.  The norms are summed from the same operands, and a point against
// itself gets distance 0 exactly.
#include <cmath>

#include "device_util.hpp"
#include "internal.hpp"

namespace invaskit {
namespace {

constexpr int ET = kEvalTile;  // 64
constexpr int DC = 8;          // coordinates per LDS chunk

// exp(a) for a kernel value stored as T (a = -|x-y|^2 / (2h^2) <= 0, from
// FP64 distances): FP64 exp for FP64 blocks; for FP32 blocks the FP32 exp of
// the rounded argument, whose absolute error, at most about u32 max(a e^a)
// = u32 / e, is below the FP32 rounding of values near 1/e, at a fraction
// of the cost of the FP64 exp
template <typename T>
__device__ __forceinline__ double kernel_value(double a) {
  if constexpr (sizeof(T) == 4)
    return (double)expf((float)a);
  else
    return exp(a);
}

template <typename PT, typename T>
__global__ __launch_bounds__(256) void k_eval(const PT* __restrict__ X, int d, double nhalf_inv_h2,
                                              double shift, const EvalBlock* __restrict__ blocks,
                                              const Tile3* __restrict__ tiles) {
  __shared__ double xr[DC][ET + 1];
  __shared__ double xc[DC][ET + 1];
  __shared__ int64_t cidx[ET];
  const Tile3 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const EvalBlock b = blocks[t.prob];
  const int r0 = t.tm * ET, c0 = t.tn * ET;
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;

  if (tid < ET) {
    const int c = c0 + tid;
    int64_t g = -1;
    if (c < b.ncols) g = b.cols ? (int64_t)glb(b.cols)[c] : b.col0 + c;
    cidx[tid] = g;
  }
  __syncthreads();

  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int dd = 0; dd < d; dd += DC) {
    // all of a thread's coordinate loads are issued before any is staged
    // (indices past the tile read its first point and are zeroed)
    constexpr int PER = ET * DC / 256;
    double vr[PER], vc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + 256 * q;
      const int p = idx / DC, k = idx % DC;
      const int kk = min(dd + k, d - 1);
      const int r = r0 + p;
      vr[q] = (double)X[(b.row0 + (r < b.rows ? r : 0)) * d + kk];
      const int64_t g = cidx[p];
      vc[q] = (double)X[(g >= 0 ? g : b.row0) * d + kk];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + 256 * q;
      const int p = idx / DC, k = idx % DC;
      const bool kin = dd + k < d;
      xr[k][p] = (r0 + p < b.rows && kin) ? vr[q] : 0.0;
      xc[k][p] = (cidx[p] >= 0 && kin) ? vc[q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DC; ++k) {
      double a[4], c[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = xr[k][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = xc[k][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double df = a[i] - c[j];
          acc[i][j] = fma(df, df, acc[i][j]);
        }
    }
    __syncthreads();
  }

  const gptr<T> out = glb(static_cast<T*>(b.out));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = c0 + tc + 16 * j;
    if (c >= b.ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + tr + 16 * i;
      if (r >= b.rows) continue;
      double v = kernel_value<T>(acc[i][j] * nhalf_inv_h2);
      if (b.diag && r == c) v += shift;
      out[(int64_t)c * b.ld + r] = (T)v;
    }
  }
}

// ---------------------------------------------------------------- Gram form
constexpr int GK = 32;       // coordinates per LDS stage
constexpr int GKP = GK + 4;  // LDS row stride (spreads the operand reads over the banks)

// The 64 x 64 Gram tile G[c][r] = (y_c - z) . (x_r - z), z = X[ref], over
// all d coordinates in FP64: row points rowi[p] and column points coli[p]
// (LDS, -1 for none: zero operands), staged GK coordinates at a time through
// sr / sc with the next stage prefetched into registers.  Wave w holds rows
// 32 (w & 1) .. +32 and columns 32 (w >> 1) .. +32 as 2 x 2 MFMA 16 x 16
// tiles, the MFMA row index being the column point c (so the lanes of an
// accumulator run along r).  Threads 0..63 also return the squared norm of
// row point tid, threads 64..127 that of column point tid - 64.  Starts and
// ends with a barrier.
template <typename PT>
__device__ __forceinline__ void gram_tile(const PT* __restrict__ X, int d, int64_t ref,
                                          const int64_t* rowi, const int64_t* coli,
                                          double (*sr)[GKP], double (*sc)[GKP],
                                          f64x4 (&acc)[2][2], double& nrm) {
  using T = double;
  using V4 = f64x4;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wr = wave & 1, wc = wave >> 1;
  const int k = tid % GK;   // this thread's coordinate within a stage
  const int p0 = tid / GK;  // and its points p0 + 8 i
  constexpr int NP = 64 * GK / 256;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  nrm = 0.0;
  __syncthreads();  // rowi / coli written by the caller
  T vr[NP], vc[NP];
  auto load = [&](int dd) {
    const int kk = dd + k;
    const bool kin = kk < d;
    const double z = kin ? (double)X[ref * d + kk] : 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int64_t gr = rowi[p0 + 8 * i], gc = coli[p0 + 8 * i];
      vr[i] = (gr >= 0 && kin) ? (double)X[gr * d + kk] - z : 0.0;
      vc[i] = (gc >= 0 && kin) ? (double)X[gc * d + kk] - z : 0.0;
    }
  };
  load(0);
  for (int dd = 0; dd < d; dd += GK) {
    __syncthreads();  // the previous stage's operands are consumed
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      sr[p0 + 8 * i][k] = vr[i];
      sc[p0 + 8 * i][k] = vc[i];
    }
    __syncthreads();
    if (dd + GK < d) load(dd + GK);
    if (tid < 128) {
      const T* q = tid < 64 ? sr[tid] : sc[tid - 64];
#pragma unroll
      for (int kq = 0; kq < GK; ++kq) nrm = fma(q[kq], q[kq], nrm);
    }
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      T a[2], b[2];
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) a[ci] = sc[32 * wc + 16 * ci + lr][4 * ks + lg];
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) b[ri] = sr[32 * wr + 16 * ri + lr][4 * ks + lg];
#pragma unroll
      for (int ci = 0; ci < 2; ++ci)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) acc[ci][ri] = mfma16(a[ci], b[ri], acc[ci][ri]);
    }
  }
  __syncthreads();
}

// k_eval for d > 64: the same 64 x 64 tiles and stores, distances in the Gram
// form on the matrix cores (FP64), kernel values stored in T.
template <typename PT, typename T>
__global__ __launch_bounds__(256) void k_eval_gram(const PT* __restrict__ X, int d,
                                                   double nhalf_inv_h2, double shift,
                                                   const EvalBlock* __restrict__ blocks,
                                                   const Tile3* __restrict__ tiles) {
  __shared__ double sr[ET][GKP];
  __shared__ double sc[ET][GKP];
  __shared__ int64_t rowi[ET], coli[ET];
  __shared__ double nr[ET], nc[ET];
  const Tile3 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const EvalBlock b = blocks[t.prob];
  const int r0 = t.tm * ET, c0 = t.tn * ET;
  const int tid = threadIdx.x;
  if (tid < ET) {
    const int r = r0 + tid;
    rowi[tid] = (r < b.rows) ? b.row0 + r : -1;
  } else if (tid < 2 * ET) {
    const int c = c0 + tid - ET;
    int64_t g = -1;
    if (c < b.ncols) g = b.cols ? (int64_t)glb(b.cols)[c] : b.col0 + c;
    coli[tid - ET] = g;
  }
  f64x4 acc[2][2];
  double nrm;
  gram_tile<PT>(X, d, b.row0 + r0, rowi, coli, sr, sc, acc, nrm);
  if (tid < ET)
    nr[tid] = nrm;
  else if (tid < 2 * ET)
    nc[tid - ET] = nrm;
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wr = wave & 1, wc = wave >> 1;
  const gptr<T> out = glb(static_cast<T*>(b.out));
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
    const int rl = 32 * wr + 16 * ri + lr;
    const int r = r0 + rl;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cl = 32 * wc + 16 * ci + acc_row(0.0, lg, v);
        const int c = c0 + cl;
        if (r < b.rows && c < b.ncols) {
          double r2 = fmax(nr[rl] + nc[cl] - 2.0 * acc[ci][ri][v], 0.0);
          if (rowi[rl] == coli[cl]) r2 = 0.0;
          double val = kernel_value<T>(r2 * nhalf_inv_h2);
          if (b.diag && r == c) val += shift;
          out[(int64_t)c * b.ld + r] = (T)val;
        }
      }
  }
}

// exp(a) for a <= 0 by Tang's table-driven method (ACM TOMS 15(2), 1989).
// With n = round(64 a / ln 2) = 64 k + j (0 <= j < 64) and
// r = a - n ln2/64, |r| <= ln2/128, exp(a) = 2^k 2^(j/64) e^r.  ln2/64 is
// split in two so that n times its leading part is exact; e^r - 1 is its
// degree-5 Taylor polynomial, whose truncation error at |r| = ln2/128 is
// below 4e-17; tab holds 2^(j/64).  The result is within about two units
// in the last place of exp(a), in 14 vector operations and one LDS read
// instead of the library's 22.  Arguments below -800 give 0, as exp does;
// the method holds as well for the small positive arguments that rounding
// can leave where the exact exponent is 0.
__device__ __host__ __forceinline__ double exp_nonpos(double a, const double* tab) {
  constexpr double kInvL = 0x1.71547652b82fep+6;  // 64 / ln 2
  constexpr double kLhi = 0x1.62e42fee00000p-7;   // ln 2 / 64, leading 32 bits
  constexpr double kLlo = 0x1.a39ef35793c76p-39;  // ln 2 / 64 - kLhi
  a = fmax(a, -800.0);
  const double n = rint(a * kInvL);
  const double r = fma(-n, kLlo, fma(-n, kLhi, a));
  const int ni = (int)n;
  const double t = tab[ni & 63];
  const double p = r * fma(r, fma(r, fma(r, fma(r, 1.0 / 120, 1.0 / 24), 1.0 / 6), 0.5), 1.0);
  return ldexp(fma(t, p, t), ni >> 6);
}

constexpr int MB = kMvBlock;  // targets per workgroup
constexpr int MS = 64;        // sources per LDS stage
// RC right-hand sides per pass over the sources: 4, or 16 when there are
// more than 4, so that every kernel value serves 16 columns and the
// distances are computed a quarter as often (the Gram form keeps 4: its
// registers also hold the MFMA tiles)

// TPT targets per thread (2 for d <= 16: two independent distance/exp
// chains per thread and half the LDS reads per pair), MB / TPT threads.
// Source rows are read by all lanes at once (LDS broadcast), so they are
// stored unpadded and read as 16-byte vectors.
template <typename PT, int DM, int TPT, int RC>
__global__ __launch_bounds__(MB / TPT) void k_mv_eval(const PT* __restrict__ X, int d,
                                                      double nhalf_inv_h2, double lam,
                                                      const MvTile* __restrict__ tiles,
                                                      const MvSeg* __restrict__ segs,
                                                      const double* __restrict__ x, int64_t ldx,
                                                      double* __restrict__ y, int64_t ldy,
                                                      const double* __restrict__ bsub, int64_t ldb,
                                                      int nrhs, int mode) {
  constexpr int NT = MB / TPT;
  constexpr int LIT = (MS * DM + NT - 1) / NT;  // source coordinates per thread and stage
  constexpr int LCH = LIT < 4 ? LIT : 4;        // of them loaded together
  static_assert(LIT % LCH == 0, "stage loads in whole chunks");
  __shared__ __align__(16) double sx[MS][DM];  // source coordinates minus z
  __shared__ double sn[MS];                    // c |y - z|^2 of each source
  __shared__ __align__(16) double sw[MS][RC];
  __shared__ double s_tab[64];  // 2^(j/64) for exp_nonpos
  const MvTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const int tid = threadIdx.x;
  if (tid < 64) s_tab[tid] = exp2((double)tid * (1.0 / 64));  // before the first stage's barrier
  // Exponent c |x - y|^2 (c = -1/(2h^2)) in the shifted Gram form
  // c |x'|^2 + c |y'|^2 + (-2c) x'.y', x' = x - z, y' = y - z, z the tile's
  // first target: one product per coordinate instead of a difference and a
  // product.  The shift keeps |x'|, |y'| at the scale of the distances
  // between a leaf's points, so the rounding of the exponent stays near
  // the unit roundoff times the squared distances; far sources give
  // exponents whose kernel values are negligible anyway.
  __shared__ double zc[DM];
  if (tid < DM) zc[tid] = (tid < d) ? (double)X[(int64_t)t.row0 * d + tid] : 0.0;
  __syncthreads();
  const double m2c = -2.0 * nhalf_inv_h2;
  double xi[TPT][DM], cx[TPT];
  // the targets' coordinates: every load issued before the first is used
  // (rows and coordinates clamped into range, masked afterwards), so that
  // they are in flight together instead of one after another
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int64_t rr = t.row0 + min(tid + NT * u, t.rows - 1);
#pragma unroll
    for (int k = 0; k < DM; ++k) xi[u][k] = (double)X[rr * d + min(k, d - 1)];
  }
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const bool active = tid + NT * u < t.rows;
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < DM; ++k) {
      const double v = (active && k < d) ? xi[u][k] - zc[k] : 0.0;
      nrm = fma(v, v, nrm);
      xi[u][k] = m2c * v;
    }
    cx[u] = nhalf_inv_h2 * nrm;
  }

  for (int cb = 0; cb < nrhs; cb += RC) {
    const int ncol = min(RC, nrhs - cb);
    double acc[TPT][RC];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int r = tid + NT * u;
#pragma unroll
      for (int c = 0; c < RC; ++c)
        acc[u][c] = (mode == kMvFar && r < t.rows && c < ncol)
                        ? y[(int64_t)(cb + c) * ldy + t.row0 + r]
                        : 0.0;
    }
    const int s_lo = t.seg0 + (mode == kMvFar ? 1 : 0);
    const int s_hi = mode == kMvNear ? t.seg0 + 1 : t.seg0 + t.nseg;
    for (int s = s_lo; s < s_hi; ++s) {
      const MvSeg g = segs[s];
      for (int j0 = 0; j0 < g.count; j0 += MS) {
        const int nj = min(MS, g.count - j0);
        __syncthreads();
        // the stage's source coordinates, LCH loads in flight at a time:
        // first their point indices, then the coordinates (sources and
        // coordinates clamped into range, masked when stored)
        for (int i0 = 0; i0 < LIT; i0 += LCH) {
          int64_t pp[LCH];
          double xv[LCH];
          if (g.idx) {  // (uniform: one branch around all the index loads)
            const gptr<const int32_t> gi = glb(g.idx) + j0;
#pragma unroll
            for (int u = 0; u < LCH; ++u) pp[u] = gi[min((tid + NT * (i0 + u)) / DM, nj - 1)];
          } else {
#pragma unroll
            for (int u = 0; u < LCH; ++u)
              pp[u] = g.p0 + j0 + min((tid + NT * (i0 + u)) / DM, nj - 1);
          }
#pragma unroll
          for (int u = 0; u < LCH; ++u)
            xv[u] = (double)X[pp[u] * d + min((tid + NT * (i0 + u)) % DM, d - 1)];
#pragma unroll
          for (int u = 0; u < LCH; ++u) {
            const int idx = tid + NT * (i0 + u);
            const int j = idx / DM, k = idx % DM;
            if (idx < MS * DM) sx[j][k] = (j < nj && k < d) ? xv[u] - zc[k] : 0.0;
          }
        }
        for (int idx = tid; idx < MS * RC; idx += NT) {
          const int j = idx / RC, c = idx % RC;
          const double v =
              glb(g.w)[(int64_t)(cb + min(c, ncol - 1)) * g.ldw + j0 + min(j, nj - 1)];
          sw[j][c] = (j < nj && c < ncol) ? v : 0.0;
        }
        __syncthreads();
        if (tid < MS) {
          double nrm = 0.0;
#pragma unroll
          for (int k = 0; k < DM; ++k) nrm = fma(sx[tid][k], sx[tid][k], nrm);
          sn[tid] = nhalf_inv_h2 * nrm;
        }
        __syncthreads();
        for (int j = 0; j < nj; ++j) {
          double wv[RC];
#pragma unroll
          for (int c = 0; c < RC; ++c) wv[c] = sw[j][c];
          // two targets share one register copy of the source row; a single
          // target reads it from LDS as it goes (a wide row would not fit)
          double sv[TPT > 1 ? DM : 1];
          if constexpr (TPT > 1) {
#pragma unroll
            for (int k = 0; k < DM; ++k) sv[k] = sx[j][k];
          }
          const double cy = sn[j];
#pragma unroll
          for (int u = 0; u < TPT; ++u) {
            // the exponent; rounding can leave it a little above 0, where
            // exp_nonpos stays accurate
            double e = cx[u] + cy;
#pragma unroll
            for (int k = 0; k < DM; ++k) {
              if constexpr (TPT > 1)
                e = fma(xi[u][k], sv[k], e);
              else
                e = fma(xi[u][k], sx[j][k], e);
            }
            const double kv = exp_nonpos(e, s_tab);
#pragma unroll
            for (int c = 0; c < RC; ++c) acc[u][c] = fma(kv, wv[c], acc[u][c]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int r = tid + NT * u;
      if (r < t.rows) {
        const int64_t i = t.row0 + r;
        // unrolled over RC (guarded by ncol) so that acc stays in registers:
        // a loop bound known only at run time would index it dynamically
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          if (c >= ncol) continue;
          if (mode == kMvNear) {
            y[(int64_t)(cb + c) * ldy + i] = acc[u][c];
            continue;
          }
          const double ax = lam * x[(int64_t)(cb + c) * ldx + i] + acc[u][c];
          y[(int64_t)(cb + c) * ldy + i] = bsub ? bsub[(int64_t)(cb + c) * ldb + i] - ax : ax;
        }
      }
    }
  }
}

constexpr int WT = kMvWideRows;  // targets per workgroup of the d > 64 form
constexpr int WS = 64;           // sources per stage

// k_mv_eval for d > 64, in the Gram form (FP64 MFMA): a workgroup takes 64 targets
// against 64 sources at a time; each lane turns its Gram entries into kernel
// values and accumulates K w for its targets over the sources it holds; at
// the end the four lane groups of a target are summed across lanes and the
// two waves that share it through LDS.
template <typename PT, int RC>
__global__ __launch_bounds__(256) void k_mv_eval_gram(
    const PT* __restrict__ X, int d, double nhalf_inv_h2, double lam,
    const MvTile* __restrict__ tiles, const MvSeg* __restrict__ segs,
    const double* __restrict__ x, int64_t ldx, double* __restrict__ y, int64_t ldy,
    const double* __restrict__ bsub, int64_t ldb, int nrhs) {
  __shared__ double sr[WT][GKP];
  __shared__ double sc[WS][GKP];
  __shared__ int64_t rowi[WT], coli[WS];
  __shared__ double nr[WT], nc[WS];
  __shared__ double sw[WS][RC];
  __shared__ double red[2][WT][RC];
  const MvTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wr = wave & 1, wc = wave >> 1;
  if (tid < WT) rowi[tid] = (tid < t.rows) ? t.row0 + tid : -1;

  for (int cb = 0; cb < nrhs; cb += RC) {
    const int ncol = min(RC, nrhs - cb);
    double acc[2][RC];
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int c = 0; c < RC; ++c) acc[ri][c] = 0.0;
    for (int sg = t.seg0; sg < t.seg0 + t.nseg; ++sg) {
      const MvSeg g = segs[sg];
      for (int j0 = 0; j0 < g.count; j0 += WS) {
        const int nj = min(WS, g.count - j0);
        __syncthreads();  // the previous stage's coli, sw, nr, nc are consumed
        if (tid < WS)
          coli[tid] = (tid < nj) ? (g.idx ? (int64_t)glb(g.idx)[j0 + tid] : g.p0 + j0 + tid) : -1;
        for (int idx = tid; idx < WS * RC; idx += 256) {
          const int j = idx / RC, c = idx % RC;
          sw[j][c] = (j < nj && c < ncol) ? glb(g.w)[(int64_t)(cb + c) * g.ldw + j0 + j] : 0.0;
        }
        f64x4 gm[2][2];
        double nrm;
        gram_tile<PT>(X, d, t.row0, rowi, coli, sr, sc, gm, nrm);
        if (tid < WT)
          nr[tid] = nrm;
        else if (tid < WT + WS)
          nc[tid - WT] = nrm;
        __syncthreads();
        // sources past nj carry zero weight
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          const int rl = 32 * wr + 16 * ri + lr;
#pragma unroll
          for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int cl = 32 * wc + 16 * ci + acc_row(0.0, lg, v);
              double r2 = fmax(nr[rl] + nc[cl] - 2.0 * gm[ci][ri][v], 0.0);
              if (rowi[rl] == coli[cl]) r2 = 0.0;
              const double kv = exp(r2 * nhalf_inv_h2);
#pragma unroll
              for (int c = 0; c < RC; ++c) acc[ri][c] = fma(kv, sw[cl][c], acc[ri][c]);
            }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        double v = acc[ri][c];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lg == 0) red[wc][32 * wr + 16 * ri + lr][c] = v;
      }
    __syncthreads();
    if (tid < t.rows) {
      const int64_t i = t.row0 + tid;
      for (int c = 0; c < ncol; ++c) {
        const double sum = red[0][tid][c] + red[1][tid][c];
        const double ax = lam * x[(int64_t)(cb + c) * ldx + i] + sum;
        y[(int64_t)(cb + c) * ldy + i] = bsub ? bsub[(int64_t)(cb + c) * ldb + i] - ax : ax;
      }
    }
  }
}

}  // namespace

template <typename PT, typename T>
hipError_t launch_eval(const PT* X, int d, double h, double shift, const EvalBlock* blocks,
                       const Tile3* tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const double c = -0.5 / (h * h);
  if (d > kMvMaxDim)
    hipLaunchKernelGGL((k_eval_gram<PT, T>), dim3(ntiles), dim3(256), 0, s, X, d, c, shift,
                       blocks, tiles);
  else
    hipLaunchKernelGGL((k_eval<PT, T>), dim3(ntiles), dim3(256), 0, s, X, d, c, shift, blocks,
                       tiles);
  return hipGetLastError();
}

template <typename PT>
hipError_t launch_mv_eval(const PT* X, int d, double h, double lam, const MvTile* tiles,
                          int ntiles, const MvSeg* segs, const double* x, int64_t ldx,
                          double* y, int64_t ldy, const double* b, int64_t ldb, int nrhs,
                          int mode, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (mode != kMvWhole && d > kMvMaxDim) return hipErrorInvalidValue;
  const double c = -0.5 / (h * h);
#define INVASKIT_MV(DMV, RCV)                                                                \
  hipLaunchKernelGGL((k_mv_eval<PT, DMV, (DMV <= 16 ? 2 : 1), RCV>), dim3(ntiles),          \
                     dim3(MB / (DMV <= 16 ? 2 : 1)), 0, s, X, d, c, lam, tiles, segs, x, ldx, y, \
                     ldy, b, ldb, nrhs, mode)
#define INVASKIT_MV_RC(RCV)                                                                  \
  if (d <= 8)                                                                                \
    INVASKIT_MV(8, RCV);                                                                     \
  else if (d <= 16)                                                                          \
    INVASKIT_MV(16, RCV);                                                                    \
  else if (d <= 32)                                                                          \
    INVASKIT_MV(32, RCV);                                                                    \
  else if (d <= 64)                                                                          \
    INVASKIT_MV(64, RCV);                                                                    \
  else                                                                                       \
    hipLaunchKernelGGL((k_mv_eval_gram<PT, 4>), dim3(ntiles), dim3(256), 0, s, X, d, c, lam,   \
                       tiles, segs, x, ldx, y, ldy, b, ldb, nrhs)
  // columns per pass: one for a single right-hand side (no idle
  // accumulators), four, or sixteen
  if (nrhs == 1) {
    INVASKIT_MV_RC(1);
  } else if (nrhs <= 4) {
    INVASKIT_MV_RC(4);
  } else {
    INVASKIT_MV_RC(16);
  }
#undef INVASKIT_MV_RC
#undef INVASKIT_MV
  return hipGetLastError();
}

template hipError_t launch_eval<double, double>(const double*, int, double, double,
                                                const EvalBlock*, const Tile3*, int, hipStream_t);
template hipError_t launch_eval<double, float>(const double*, int, double, double,
                                               const EvalBlock*, const Tile3*, int, hipStream_t);
template hipError_t launch_eval<float, double>(const float*, int, double, double,
                                               const EvalBlock*, const Tile3*, int, hipStream_t);
template hipError_t launch_eval<float, float>(const float*, int, double, double,
                                              const EvalBlock*, const Tile3*, int, hipStream_t);
template hipError_t launch_mv_eval<double>(const double*, int, double, double, const MvTile*,
                                           int, const MvSeg*, const double*, int64_t, double*,
                                           int64_t, const double*, int64_t, int, int, hipStream_t);
template hipError_t launch_mv_eval<float>(const float*, int, double, double, const MvTile*, int,
                                          const MvSeg*, const double*, int64_t, double*, int64_t,
                                          const double*, int64_t, int, int, hipStream_t);

}  // namespace invaskit
