// Internal interfaces of libinvaskit: work descriptors consumed by the
// batched HIP kernels and the host launchers that enqueue them.
//
// Every batched kernel reads a device-resident table of problems ("probs")
// plus a table of work tiles; one workgroup handles one tile.  The tables are
// built on the host when a factorization is planned and uploaded once, so
// each launch only passes table pointers and a tile count.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace invaskit {

// C[M x N] = beta * C + alpha * sum_s A_s B_s.  B_s is column-major
// (k x N, ldb); A_s is column-major (M x k, lda) or row-major when a_rm.
// C is column-major (ldc).  beta == 0 never reads C.
struct GemmSeg {
  const void* A;
  const void* B;
  int64_t lda, ldb;
  int32_t k;
  int32_t a_rm;
};

struct GemmProb {
  void* C;
  int64_t ldc;
  int32_t M, N;
  int32_t seg0, nseg;
  double alpha, beta;
};

// Grouped GEMM tiles: kGemmTileM rows (four waves of 32) by up to
// kGemmMaxCols columns.  A product with N <= kGemmMaxCols is one column
// tile of width 16 * ceil(N / 16); wider products are cut into tiles of
// kGemmColChunk columns.
constexpr int kGemmTileM = 128;
constexpr int kGemmMaxCols = 80;
constexpr int kGemmColChunk = 64;

struct Tile3 {
  int32_t prob, tm, tn;
};

struct Tile2 {
  int32_t prob, tn;
};

// In-place style triangular solve with an LU factor (row permutation, unit
// lower L, upper U; the factor is stored row-major).  Right-hand-side rows [0, split) come from in0 (ldin0),
// rows [split, n) from in1 (ldin1); the solution goes to out (ldout).  Input
// and output may be the same buffer.
struct TrsmProb {
  const void* lu;
  const void* dinv;  // inverses of the 64 x 64 diagonal blocks (k_diag_inv layout)
  const int32_t* perm;
  int32_t n, nrhs;
  const void* in0;
  const void* in1;
  int64_t ldin0, ldin1;
  int32_t split, pad;
  void* out;
  int64_t ldout;
};

// One 64 x 64 diagonal block of a row-major LU factor (rows/columns
// jb .. jb+63): out receives inv(L_bb) then inv(U_bb), each 64 x 64
// row-major, zero beyond the matrix order.
struct DiagInvProb {
  const void* lu;
  const int32_t* perm;  // factor row j is stored in row perm[j]
  void* out;
  int32_t n, jb;
};
constexpr int kDiagBlock = 64;
constexpr int kLdsBytes = 160 * 1024;  // LDS of one compute unit

struct LuProb {
  void* a;
  int32_t* perm;
  int32_t* info;
  int32_t n, pad;
};

// out[r + c*ld] = K(x[row0 + r], x[col(c)]) (+ shift on the diagonal when
// diag != 0); col(c) = cols ? cols[c] : col0 + c.
struct EvalBlock {
  void* out;
  int64_t ld;
  int64_t row0;
  const int32_t* cols;
  int64_t col0;
  int32_t rows, ncols;
  int32_t diag, pad;
};

// Reduced system Z (n = sr + sl, row-major) = [[I, pr], [pl, I]] with
// pr: sr x sl (ld sr) and pl: sl x sr (ld sl).
struct ZformProb {
  void* Z;
  const void* pr;
  const void* pl;
  int32_t sr, sl;
};

// dst = src + shift * I, square blocks of order m (the leaf blocks of one
// factorization of a lambda sweep, copied from the shared lambda-free ones)
struct CopyShiftProb {
  const void* src;
  void* dst;
  int32_t m, pad;
  double shift;
};

// Fused FP64 kernel-times-weights evaluation for one block of targets:
// y[i] (+)= sum over segments of sum_j K(x_i, x_src(j)) w[j, :].
struct MvSeg {
  const int32_t* idx;  // source point ids, or nullptr for p0 + j
  int64_t p0;
  const double* w;
  int64_t ldw;
  int32_t count, pad;
};

struct MvTile {
  int64_t row0;  // first target point
  int32_t rows;  // targets in this tile (<= block size)
  int32_t seg0, nseg, pad;
};

// Workgroup -> tile mapping that keeps runs of consecutive tiles on one XCD.
// The hardware places workgroup b on XCD b % 8; each XCD has its own L2.
// Tile tables list the tiles of one problem (one leaf, one node)
// consecutively, so a run of kXcdRun tiles on one XCD shares the problem's
// operands in that L2.  The runs themselves are dealt round-robin, so the
// XCDs stay balanced when tile cost drifts along the table (leaf sizes follow
// the tree's random splits).  Tiles past the last whole round of runs keep
// the hardware order.  Bijective for any grid size.
constexpr int kXcds = 8;
constexpr int kXcdRun = 8;
__device__ __host__ __forceinline__ int xcd_tile(int b, int nb) {
  const int full = nb / (kXcds * kXcdRun) * (kXcds * kXcdRun);
  if (b >= full) return b;
  const int x = b % kXcds, slot = b / kXcds;
  return ((slot / kXcdRun) * kXcds + x) * kXcdRun + slot % kXcdRun;
}

// ---------------------------------------------------------------- launchers
// transposed: the problems of this tile list compute C^T row-major (C stored
// row-major with row stride ldc); otherwise C is column-major
template <typename T>
hipError_t launch_gemm(const GemmProb* probs, const GemmSeg* segs, const Tile3* tiles,
                       int ntiles, bool transposed, hipStream_t s);
// skinny forms, one workgroup per problem, every N <= kGemvCols:
// kGemvSplitK: M <= kGemvRows, A column-major, the four waves split K;
// kGemvRowMajor: A row-major, one wave per row (chosen for a mean K of at
// least kGemvRmMinK)
constexpr int kGemvCols = 4;
constexpr int kGemvRows = 128;
constexpr int kGemvRmMinK = 128;
constexpr int kGemvSplitK = 1, kGemvRowMajor = 3;
// kGemvTall: A column-major, M above kGemvRows: workgroups of kGemvTallRows
// rows listed in a tile table (Tile3: prob, tm), four consecutive rows per
// lane (one 16-byte load per column), the four waves splitting K
constexpr int kGemvTall = 4;
constexpr int kGemvTallRows = 256;
template <typename T>
hipError_t launch_gemv_tall(const GemmProb* probs, const GemmSeg* segs, const Tile3* tiles,
                            int ntiles, hipStream_t s);
template <typename T>
hipError_t launch_gemv(const GemmProb* probs, const GemmSeg* segs, int count, int form,
                       hipStream_t s);

// kind: 0 leaf panels of the factorization, 1 reduced systems, 2 solve phase
// (library factors, padded by 64 elements), 3 caller-owned factors.  cols:
// right-hand sides per workgroup, 16 or 32 (tile tn covers columns
// [tn cols, (tn+1) cols)); hipErrorInvalidValue if the workgroup's LDS,
// getrs_lds_bytes(nmax, sizeof(TZ), cols), exceeds kLdsBytes.
template <typename TZ, typename TV>
hipError_t launch_getrs(const TrsmProb* probs, const Tile2* tiles, int ntiles, int nmax, int kind,
                        int cols, hipStream_t s);
size_t getrs_lds_bytes(int nmax, size_t tz_bytes, int cols);
constexpr int kTrsmColsDefault = 16;
template <typename TZ>
hipError_t launch_diag_inv(const DiagInvProb* probs, int count, hipStream_t s);

// kind: 0 leaf blocks, 1 reduced systems.  panel: the LU panel width, 0 for
// the default (getrf_default_panel), or 16 / 32 for kind 0; waves: waves per
// matrix of the block kernel, 0 for the default (4), or 4 / 8 for kind 0.
// form (orders up to kOneWaveMax): kLuFormAuto takes the one-wave kernel in
// FP32 and the block kernel in FP64; kLuFormOneWave and kLuFormBlock force
// one of them.  nopiv (kind 0, block kernel): no row exchanges, for
// symmetric positive definite blocks; info then flags the first pivot that
// is not positive and finite.
constexpr int kLuFormAuto = 0, kLuFormOneWave = 1, kLuFormBlock = 2;
constexpr int kOneWaveMax = 192;
template <typename T>
hipError_t launch_getrf(const LuProb* probs, int count, int nmax, int kind, int panel, int waves,
                        hipStream_t s, int form = kLuFormAuto, bool nopiv = false);
int getrf_default_panel(bool t64);

template <typename PT, typename T>
hipError_t launch_eval(const PT* X, int d, double h, double shift, const EvalBlock* blocks,
                       const Tile3* tiles, int ntiles, hipStream_t s);
constexpr int kEvalTile = 64;

template <typename T>
hipError_t launch_copy_shift(const CopyShiftProb* probs, int count, hipStream_t s);

template <typename TZ, typename TV>
hipError_t launch_zform(const ZformProb* probs, int count, hipStream_t s);

// y = lam*x + sum K w  (or b - that, when b != nullptr), columns [c0, c0+nc).
// mode kMvWhole sums every segment of a tile; kMvNear sums only its first
// segment (the leaf's own block) and stores the raw sum in y; kMvFar starts
// from that sum in y and adds the remaining segments, in the same order, so
// the two halves give the same bits as one kMvWhole launch.  The halves are
// for d <= kMvMaxDim only.
constexpr int kMvWhole = 0, kMvNear = 1, kMvFar = 2;
template <typename PT>
hipError_t launch_mv_eval(const PT* X, int d, double h, double lam, const MvTile* tiles,
                          int ntiles, const MvSeg* segs, const double* x, int64_t ldx,
                          double* y, int64_t ldy, const double* b, int64_t ldb, int nrhs,
                          int mode, hipStream_t s);
constexpr int kMvBlock = 128;
constexpr int kMvMaxDim = 64;    // register-resident targets up to this d
constexpr int kMvWideRows = 64;  // targets per tile of the d > kMvMaxDim form

// elementwise helpers
hipError_t launch_convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s);
// out[i + c*ldo] = (TO) (in[i + c*ldi] * scale[c])  (scale may be nullptr = 1)
template <typename TI, typename TO>
hipError_t launch_copy_cols(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t n,
                            int ncols, const double* scale, bool invert_scale, hipStream_t s);
// scale[c] = sqrt(norm2[c]), c < ncols
hipError_t launch_sqrt_cols(const double* norm2, double* scale, int ncols, hipStream_t s);
// x[i + c*ldx] += scale[c] * d[i + c*ldd]
template <typename TD>
hipError_t launch_axpy_cols(double* x, int64_t ldx, const TD* d, int64_t ldd, int64_t n,
                            int ncols, const double* scale, hipStream_t s);
// v[i + c*ld] *= scale[c] (scale on the device); v[i + c*ld] = 0
hipError_t launch_scale_cols(double* v, int64_t ld, int64_t n, int ncols, const double* scale,
                             hipStream_t s);
hipError_t launch_zero_cols(double* v, int64_t ld, int64_t n, int ncols, hipStream_t s);
// out[k * ncols + c] = sum_i V_k[i, c] w[i, c] for k < nk, c < ncols, with
// V_k = V + k * vstride and column c at + c * ldv (w: + c * ldw); two
// passes through part (dots_part_doubles(n, nk, ncols) doubles), summed in
// a fixed order
size_t dots_part_doubles(int64_t n, int nk, int ncols);
hipError_t launch_dots(const double* V, int64_t vstride, int64_t ldv, int nk, const double* w,
                       int64_t ldw, int64_t n, int ncols, double* part, double* out,
                       hipStream_t s);
// out[i, c] += alpha * sum_k coef[k * ncols + c] V_k[i, c]  (coef on the device)
hipError_t launch_lincomb(double* out, int64_t ldo, const double* V, int64_t vstride,
                          int64_t ldv, int nk, const double* coef, int ncols, double alpha,
                          int64_t n, hipStream_t s);


}  // namespace invaskit
