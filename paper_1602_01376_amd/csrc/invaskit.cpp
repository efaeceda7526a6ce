// libinvaskit host side: input validation, the memory plan over the caller's
// workspace, the level-synchronous launch schedule and the C ABI of
// include/invaskit.h.
//
// Factorization (Algorithm 1), bottom-up, each step one batched launch over
// every node it touches instead of a recursion.  Notation: L = depth, c' =
// sibling of c, anc_k(i) = level-k ancestor, W^(k) = the rows of
// (lambda I + K~_cc)^-1 K(X_c, X_{c'~}) for the level-k nodes c.
//   F1  every leaf block lambda*I + K_aa is evaluated, LU-factored, and the
//       64 x 64 diagonal blocks of its factors are inverted;
//   F2  for every leaf and every level k = L .. 1 at once, the leaf's rows of
//       the skeleton block K(X_c, X_{c'~}), c = anc_k(leaf), are written
//       into the leaf-major W storage;
//   F3  every leaf applies its LU to all those columns and projects them
//       onto its skeleton, p = P_{leaf~ leaf} v;
//   F4  wavefront over the levels j = L-1 .. 0: the reduced systems
//       Z_a = I + V_a W_a of the level-j nodes are assembled from their
//       children's projections (eq. (11)), LU-factored and their diagonal
//       blocks inverted; then, for j >= 1, the skeleton sweep of level j for
//       every factor level k <= j at once:
//       y_a = Z_a^-1 [p_r; p_l] and p_a = P_{a~[l~ r~]} [y_l; y_r];
//
// F3-F4 replace the per-node "w = v - W Z V v" of Algorithm 2 by an
// algebraically identical schedule: after that update the children's
// skeleton projections of w equal y itself (V w = V v - V W y = y because
// (I + V W) y = V v), so the projection needed one level up is
// P_{b~[l~ r~]} y (eq. (12)) and never touches N-sized data.
//
// The N-sized corrections are never applied to W.  Per leaf, the corrected
// blocks satisfy W^(k) = W~^(k) - sum_{j>k} W^(j) Y^(j,k), with W~ the
// leaf-solved skeleton blocks and Y^(j,k) blocks of the sweep solutions; in
// matrix form W = W~ (I + U)^-1 with U strictly block-triangular.  The solve
// needs only W y^, so it computes e = (I + U)^-1 y^ by forward substitution
// on skeleton-sized data, top-down over the tree (e is one block per node),
// and then x = v - W~ e.  The solve (Algorithm 2) runs: leaf solves, leaf
// projections, the sweep for j = L-1 .. 0, the top-down pass for e, and one
// grouped GEMM per leaf.
//
// Memory.  The library allocates no device memory.  A factorization lives in
// a workspace the caller allocates (its size from
// invaskit_factor_workspace_bytes): the handle's buffers are carved from it
// at 256-byte boundaries, with the launch descriptor tables last.  A lambda
// sweep's workspace holds the lambda-free kernel blocks shared by its
// handles, the tables of its lambda-batched launches, and one region per
// handle.  Solves and products carve their vectors and tables from the
// caller's scratch.  The sizes come from the same planning code the
// factorization runs (host only, no device access), built against a
// placeholder base address: table sizes do not depend on the addresses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/invaskit.h"
#include "internal.hpp"

using namespace invaskit;

// Device scratch of invaskit_matvec_noalloc, for callers that cannot
// allocate: one copy per GPU, held until the process ends.  Host code never
// uses this name as an address: the per-device address comes from
// hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[INVASKIT_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

constexpr int kMaxLeaf = 1024;
constexpr int kMaxSkel = 512;
constexpr int kMaxDepth = 24;
constexpr int kEvents = 8;
constexpr int kPhases = 12;  // see invaskit_phase_times
constexpr size_t kAlign = 256;
// leaves of at most this order form the small class (FP32, FP64)
constexpr int kSmallLeaf32 = 192, kSmallLeaf64 = 256;
// placeholder base of the planning runs that only measure sizes; never
// dereferenced
unsigned char* const kPlanBase = reinterpret_cast<unsigned char*>(uintptr_t(1) << 40);

// -------------------------------------------------------------- small utils
// A piece of caller-owned device memory.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Assigns aligned offsets in a region, in the order pieces are taken.
struct Carve {
  size_t size = 0;
  size_t take(size_t bytes) {
    const size_t o = align_up(size, kAlign);
    size = o + std::max<size_t>(bytes, 1);
    return o;
  }
  size_t total() const { return align_up(size, kAlign); }
};

// Host staging area for descriptor tables; uploaded to one device buffer.
struct Arena {
  std::vector<unsigned char> host;
  template <typename T>
  size_t add(const std::vector<T>& v) {
    const size_t off = align_up(host.size(), kAlign);
    host.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  size_t bytes() const { return std::max<size_t>(align_up(host.size(), kAlign), kAlign); }
};

template <typename T>
const T* at(const Buf& b, size_t off) {
  return reinterpret_cast<const T*>(static_cast<unsigned char*>(b.p) + off);
}

// One batched launch, described by table offsets into a table buffer.
// A grouped GEMM launch: two tile lists over one problem table, products
// computed as stated (tiles) and products computed transposed (tiles_n).
struct GemmL {
  size_t probs = 0, segs = 0, tiles = 0, tiles_n = 0;
  int ntiles = 0, ntiles_n = 0;
  int gemv = 0, nprobs = 0;  // skinny launch: one workgroup per problem
};
struct TrsmL {
  size_t probs = 0, tiles = 0;
  int ntiles = 0, nmax = 0;
  int tz64 = 1, tv64 = 1;
  int kind = 0;
  int cols = kTrsmColsDefault;  // right-hand sides per workgroup
  double work = 0;              // sum of n^2 nrhs (tuning key)
};
struct LuL {
  size_t probs = 0;
  int count = 0, nmax = 0, t64 = 1, kind = 0;
  int panel = 0;    // LU panel width, 0 = the kernel's default
  int waves = 0;    // waves per matrix, 0 = the kernel's default (4)
  int form = 0;     // kLuForm*: one-wave or block kernel for small orders
  bool nopiv = false;  // leaf blocks: the block kernel without row exchanges
  double work = 0;  // sum of n^3 (tuning key)
};
struct DinvL {
  size_t probs = 0;
  int count = 0, t64 = 1;
};
struct EvalL {
  size_t blocks = 0, tiles = 0;
  int ntiles = 0, nblocks = 0;
};
struct ZformL {
  size_t probs = 0;
  int count = 0, tz64 = 1, tv64 = 1;
};
struct CopyShiftL {
  size_t probs = 0;
  int count = 0;
};

// Kernel blocks of a problem evaluated without lambda (leaf blocks K_aa and
// the skeleton blocks of every level, in the layout of the factor storage),
// shared by the handles of a lambda sweep: only the leaf LU, W and the
// reduced systems depend on lambda.  The sweep's handles also share the
// device copy of the skeleton indices and, in mixed precision, the FP32
// copy of P.  All of it lives in the sweep's workspace.
struct KernelCache {
  Buf leaf, slab, skel, P32;
  bool valid = false;
};

// The factorization schedule: leaf-level passes over every tree level at
// once, then one wavefront step per level for the reduced systems and the
// skeleton sweep.  A plan covers one or several handles (the lambdas of a
// sweep, batched into the same launches).
struct FactorPlan {
  bool cached = false;  // kernel blocks come from a KernelCache
  EvalL leaf_eval;      // leaf blocks: into the factor storage, or the cache
  CopyShiftL leaf_copy; // cached plans: cache -> factor storage, + lambda I
  // The leaves in two size classes: [0] the large ones, on the caller's
  // stream; [1] the small ones (orders up to kSmallLeaf: the one-wave LU in
  // FP32, one panel row per thread in FP64), whose LU, diagonal-block
  // inverses and solves run on the second stream beside the large leaves'
  // LU.  Each class's solves have their own LDS size and tile choice.
  LuL leaf_lu[2];
  DinvL leaf_dinv[2];
  EvalL panels;         // skeleton blocks of every level (into W storage or the cache)
  TrsmL leaf_trsm[2][2];  // [class][16 or 32 right-hand sides per workgroup]
                          // (ntiles < 0: no room in LDS)
  GemmL leaf_proj[2];   // leaf projections of every level's panel columns, by size class
  std::vector<ZformL> zform;  // index j: reduced systems of level j
  std::vector<LuL> zlu;
  std::vector<DinvL> zdinv;
  std::vector<TrsmL> zsolve;    // index j >= 1: sweep step at level j
  std::vector<TrsmL> zsolve32;  // the same with 32 right-hand sides per workgroup
  std::vector<GemmL> pgemm;
  Buf tables;                 // device copy of the descriptor tables
};

// A matvec's buffers and launches; its tables sit inside the solve's (or
// the matvec's own) table buffer.
struct MatvecPlan {
  int r = 0;
  Buf xm, q;
  std::vector<GemmL> skel;  // levels L .. 1
  size_t mv_tiles = 0, mv_segs = 0;
  int n_mv_tiles = 0;
};

// Buffers and launches of a solve with r right-hand sides, carved from the
// caller's scratch at `base`; `blob` is the host copy of the tables.
struct SolvePlan {
  int r = 0;
  bool solve = true;           // false: a matvec-only plan
  void* base = nullptr;
  size_t min_bytes = 0, full_bytes = 0;  // scratch without / with the GMRES bases
  std::vector<unsigned char> blob;
  Buf tables, xbuf, sbuf;      // xbuf/sbuf in the factor precision
  Buf x64, r64, sc;            // refinement: iterate, residual, column scales
  Buf gpart, gsmall;           // reduction partials; small per-column vectors
  Buf gmV, gmZ;                // GMRES bases (present when the scratch holds them)
  int gm_m = 0;                // Krylov vectors per GMRES cycle (0: no room)
  TrsmL leaf_trsm;
  GemmL leaf_proj;
  std::vector<TrsmL> zsolve;   // levels L-1 .. 0
  std::vector<GemmL> pgemm;    // levels L-1 .. 1
  std::vector<GemmL> topdown;  // e = (I + U)^-1 y^, levels 2 .. L
  GemmL final_;
  MatvecPlan mv;
};

}  // namespace

struct invaskit_handle_s {
  // options
  int prec = INVASKIT_PREC_FP64;
  int top64 = 4;
  double tol = 1e-10;
  int maxit = 30;
  int tune = INVASKIT_TUNE_AUTO;
  int fix_lu_panel = 0, fix_lu_waves = 0, fix_trsm_cols = 0;  // 0: chosen by tuning
  int fix_zlu_form = 0, fix_zsolve_cols = 0;                   // likewise
  int leaf_pivoting = INVASKIT_LEAF_PIVOT_AUTO;
  bool leaf_nopiv = false;  // the next factor runs the leaf LU without row exchanges
  int refine = INVASKIT_REFINE_AUTO;
  int gm_restart = 20, gm_maxit = 300;
  hipStream_t stream = nullptr;
  // problem (device data borrowed)
  int64_t N = 0;
  int d = 0, L = 0, pdt = INVASKIT_F64;
  const void* X = nullptr;
  const double* P64 = nullptr;
  double h = 1.0, lam = 0.0;
  std::vector<int64_t> leaf_off, skel_off, p_off;
  std::vector<int32_t> skel_idx;
  // derived tree data
  int nn = 0, nleaves = 0;
  std::vector<int64_t> na, nb;  // node point ranges
  std::vector<int> s, w, z;
  // layout
  std::vector<int64_t> lu_off, slab_off, z_off, zperm_off;
  std::vector<int> S;
  std::vector<std::vector<int>> colk;  // [leaf][level]
  std::vector<int> zis64;              // per level
  std::vector<std::vector<int>> colp;  // [node][k]: first column of factor level k
  std::vector<int> Ssw;                // sweep columns of a node (sum of its w over k)
  std::vector<int64_t> psw_off, ysw_off;
  std::vector<int64_t> dleaf_off, dz_off;
  int64_t z64n = 0, zTn = 0, zpn = 0, dz64n = 0, dzTn = 0, pswn = 0, yswn = 0;
  // buffers in the caller's workspace
  void* region = nullptr;  // this handle's region
  size_t region_bytes = 0;
  Buf leafLU, leafPerm, leafInfo, slab, Z64, ZT, zperm, zinfo, psw, ysw;
  Buf dinvLeaf, dinvZ64, dinvZT;  // inverses of the 64 x 64 diagonal blocks
  Buf skel_own, P32_own;          // own copies (plain handles)
  const int32_t* skd = nullptr;   // device skeleton indices (own or the sweep's)
  const void* Pf = nullptr;       // P in the factor precision
  // schedule
  FactorPlan fp;                  // this handle's own plan
  bool fp_ready = false;          // fp built and its tables uploaded
  std::shared_ptr<KernelCache> kcache;  // set for the handles of a lambda sweep
  // solve and matvec plans, most recently used first (host memory only)
  std::list<std::unique_ptr<SolvePlan>> plans;
  const void* up_base = nullptr;  // scratch whose tables are current
  const SolvePlan* up_plan = nullptr;
  double phase_ms[kPhases] = {0};
  double plan_ms = 0;  // host planning of the handle (wall clock)
  hipEvent_t ev[kEvents + 2] = {};
  bool have_events = false;
  // the factorization schedule's events ([0] timed, [1] ordering only),
  // created on first use and reused by every later factorization: creating
  // some fifty events per call held the host behind the GPU
  std::vector<hipEvent_t> fev[2];
  // fork and join of the product's two halves (created with the side stream)
  hipEvent_t mv_ev[2] = {};
  // second stream of the factorization (default priority): the skeleton
  // blocks run on it beside the leaf block evaluation and LU
  hipStream_t side = nullptr;
  // pinned host memory for the small readbacks (pivot status, column
  // norms), so that they complete with the stream instead of blocking
  void* pin = nullptr;
  size_t pin_bytes = 0;
  invaskit_tile_config tiles{};   // tile shapes of the last factor
  std::string err;

  int level(int node) const {
    int k = 0;
    while ((2 << k) - 1 <= node) ++k;
    return k;
  }
  bool is_leaf(int node) const { return level(node) == L; }
  int sib(int c) const { return (c & 1) ? c + 1 : c - 1; }
  int anc(int node, int k) const {  // ancestor of `node` at level k (<= level(node))
    const int j = level(node);
    const int idx = node - ((1 << j) - 1);
    return (1 << k) - 1 + (idx >> (j - k));
  }
  int leaf_node(int j) const { return (1 << L) - 1 + j; }
  size_t tsize() const { return prec == INVASKIT_PREC_FP64 ? 8 : 4; }
  const void* Pt() const { return Pf; }
  const void* Z(int node) const {
    const int k = level(node);
    const Buf& b = zis64[k] ? Z64 : ZT;
    return static_cast<unsigned char*>(b.p) + z_off[node] * (zis64[k] ? 8 : 4);
  }
  void* Zm(int node) { return const_cast<void*>(Z(node)); }
  const void* DZ(int node) const {  // diagonal-block inverses of a reduced system
    const int k = level(node);
    const Buf& b = zis64[k] ? dinvZ64 : dinvZT;
    return static_cast<unsigned char*>(b.p) + dz_off[node] * (zis64[k] ? 8 : 4);
  }
  const void* DL(int leaf) const {
    return static_cast<unsigned char*>(dinvLeaf.p) + dleaf_off[leaf] * tsize();
  }

  ~invaskit_handle_s() {
    if (have_events)
      for (auto& e : ev) hipEventDestroy(e);
    for (auto& pool : fev)
      for (auto& e : pool) hipEventDestroy(e);
    for (auto& e : mv_ev)
      if (e) hipEventDestroy(e);
    if (side) hipStreamDestroy(side);
    if (pin) hipHostFree(pin);
  }
};

using H = invaskit_handle_s;

namespace {

int fail_h(H* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  g_last_error = msg;
  return code;
}

#define HIP_TRY(h, ...)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (__VA_ARGS__);                                                       \
    if (e_ != hipSuccess)                                                                \
      return fail_h((h), INVASKIT_E_HIP,                                                 \
                    std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));           \
  } while (0)

// The handle's pinned host buffer, grown to at least `bytes`.  Growing it
// frees the old one, so callers reserve it while no copy into it is pending.
int host_pinned(H* h, size_t bytes, void** out) {
  if (h->pin_bytes < bytes) {
    if (h->pin) HIP_TRY(h, hipHostFree(h->pin));
    h->pin = nullptr;
    h->pin_bytes = 0;
    const size_t want = std::max(bytes, (size_t)4096);
    HIP_TRY(h, hipHostMalloc(&h->pin, want, hipHostMallocDefault));
    h->pin_bytes = want;
  }
  *out = h->pin;
  return INVASKIT_OK;
}

int check_device(H* h) {
  int dev = 0;
  HIP_TRY(h, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(h, hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail_h(h, INVASKIT_E_DEVICE,
                  std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  return INVASKIT_OK;
}

int check_workspace(H* h, const void* ws, size_t have, size_t need, const char* what) {
  if (!ws) return fail_h(h, INVASKIT_E_ARG, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
    return fail_h(h, INVASKIT_E_ARG, std::string(what) + " must be 256-byte aligned");
  if (have < need)
    return fail_h(h, INVASKIT_E_WORKSPACE,
                  std::string(what) + " holds " + std::to_string(have) + " bytes; " +
                      std::to_string(need) + " are needed");
  return INVASKIT_OK;
}

// ------------------------------------------------------------- validation
int validate(H* h, const invaskit_problem* pb, double lambda, const invaskit_options* opt) {
  if (!pb) return fail_h(h, INVASKIT_E_ARG, "problem is NULL");
  if (pb->n < 1) return fail_h(h, INVASKIT_E_ARG, "n must be >= 1");
  if (pb->d < 1) return fail_h(h, INVASKIT_E_ARG, "d must be >= 1");
  if (pb->depth < 0 || pb->depth > kMaxDepth)
    return fail_h(h, INVASKIT_E_ARG, "depth must be in [0, 24]");
  if (pb->points_dtype != INVASKIT_F64 && pb->points_dtype != INVASKIT_F32)
    return fail_h(h, INVASKIT_E_ARG, "points_dtype must be INVASKIT_F64 or INVASKIT_F32");
  if (!pb->points) return fail_h(h, INVASKIT_E_ARG, "points is NULL");
  if (!pb->leaf_offsets || !pb->skel_offsets || !pb->p_offsets)
    return fail_h(h, INVASKIT_E_ARG, "leaf_offsets, skel_offsets and p_offsets are required");
  if (!(pb->h > 0.0) || !std::isfinite(pb->h))
    return fail_h(h, INVASKIT_E_ARG, "h must be finite and > 0");
  if (!std::isfinite(lambda)) return fail_h(h, INVASKIT_E_ARG, "lambda must be finite");
  if (opt) {
    if (opt->precision != INVASKIT_PREC_FP64 && opt->precision != INVASKIT_PREC_MIXED)
      return fail_h(h, INVASKIT_E_ARG, "precision must be INVASKIT_PREC_FP64 or _MIXED");
    if (opt->fp64_top_levels < 0) return fail_h(h, INVASKIT_E_ARG, "fp64_top_levels < 0");
    if (!(opt->refine_tol > 0.0)) return fail_h(h, INVASKIT_E_ARG, "refine_tol must be > 0");
    if (opt->max_refine_iters < 1) return fail_h(h, INVASKIT_E_ARG, "max_refine_iters < 1");
    if (opt->tune != INVASKIT_TUNE_AUTO && opt->tune != INVASKIT_TUNE_OFF)
      return fail_h(h, INVASKIT_E_ARG, "tune must be INVASKIT_TUNE_AUTO or _OFF");
    auto tile_ok = [](int v) { return v == 0 || v == 16 || v == 32; };
    if (!tile_ok(opt->leaf_lu_panel) || !tile_ok(opt->leaf_trsm_cols))
      return fail_h(h, INVASKIT_E_ARG, "leaf_lu_panel and leaf_trsm_cols must be 0, 16 or 32");
    if (opt->leaf_lu_waves != 0 && opt->leaf_lu_waves != 4 && opt->leaf_lu_waves != 8)
      return fail_h(h, INVASKIT_E_ARG, "leaf_lu_waves must be 0, 4 or 8");
    if (opt->refine < INVASKIT_REFINE_AUTO || opt->refine > INVASKIT_REFINE_NONE)
      return fail_h(h, INVASKIT_E_ARG, "refine must be one of INVASKIT_REFINE_*");
    if (opt->gmres_restart < 2 || opt->gmres_restart > 64)
      return fail_h(h, INVASKIT_E_ARG, "gmres_restart must be in [2, 64]");
    if (opt->max_gmres_iters < 1) return fail_h(h, INVASKIT_E_ARG, "max_gmres_iters < 1");
    if (opt->lambda_group < 0) return fail_h(h, INVASKIT_E_ARG, "lambda_group < 0");
    if (opt->zlu_form != 0 && opt->zlu_form != INVASKIT_ZLU_ONE_WAVE &&
        opt->zlu_form != INVASKIT_ZLU_BLOCK)
      return fail_h(h, INVASKIT_E_ARG, "zlu_form must be 0, INVASKIT_ZLU_ONE_WAVE or _BLOCK");
    if (!tile_ok(opt->zsolve_cols))
      return fail_h(h, INVASKIT_E_ARG, "zsolve_cols must be 0, 16 or 32");
    if (opt->leaf_pivoting != INVASKIT_LEAF_PIVOT_AUTO &&
        opt->leaf_pivoting != INVASKIT_LEAF_PIVOT_PARTIAL)
      return fail_h(h, INVASKIT_E_ARG, "leaf_pivoting must be INVASKIT_LEAF_PIVOT_AUTO or _PARTIAL");
  }
  const int L = pb->depth;
  const int nleaves = 1 << L;
  const int nn = (1 << (L + 1)) - 1;
  const int64_t* lo = pb->leaf_offsets;
  if (lo[0] != 0 || lo[nleaves] != pb->n)
    return fail_h(h, INVASKIT_E_ARG, "leaf_offsets must start at 0 and end at n");
  for (int j = 0; j < nleaves; ++j) {
    const int64_t m = lo[j + 1] - lo[j];
    if (m < 1 || m > kMaxLeaf)
      return fail_h(h, INVASKIT_E_ARG,
                    "leaf " + std::to_string(j) + " has " + std::to_string(m) +
                        " points; leaves must hold 1.." + std::to_string(kMaxLeaf));
  }
  const int64_t* so = pb->skel_offsets;
  if (so[0] != 0 || so[1] != 0) return fail_h(h, INVASKIT_E_ARG, "the root must have no skeleton");
  for (int c = 1; c < nn; ++c) {
    const int64_t sc = so[c + 1] - so[c];
    if (sc < 1 || sc > kMaxSkel)
      return fail_h(h, INVASKIT_E_ARG,
                    "node " + std::to_string(c) + " has " + std::to_string(sc) +
                        " skeleton points; allowed 1.." + std::to_string(kMaxSkel));
  }
  if (L > 0 && (!pb->skel_index || !pb->p_values))
    return fail_h(h, INVASKIT_E_ARG, "skel_index and p_values are required when depth > 0");
  const int64_t* po = pb->p_offsets;
  if (po[0] != 0 || po[1] != 0) return fail_h(h, INVASKIT_E_ARG, "the root has no P");
  // node ranges, nesting and P sizes
  auto range = [&](int c, int64_t& a, int64_t& b) {
    int k = 0;
    while ((2 << k) - 1 <= c) ++k;
    const int idx = c - ((1 << k) - 1);
    const int span = 1 << (L - k);
    a = lo[idx * span];
    b = lo[(idx + 1) * span];
  };
  // nesting: stamp[i] = c marks the children's skeleton points of node c
  std::vector<int32_t> stamp(L > 0 ? pb->n : 0, -1);
  for (int c = nn - 1; c >= 1; --c) {
    int64_t a, b;
    range(c, a, b);
    const int64_t sc = so[c + 1] - so[c];
    const bool leaf = (c >= (1 << L) - 1);
    int64_t cols;
    if (leaf) {
      cols = b - a;
      for (int64_t t = so[c]; t < so[c + 1]; ++t)
        if (pb->skel_index[t] < a || pb->skel_index[t] >= b)
          return fail_h(h, INVASKIT_E_ARG,
                        "skeleton of leaf node " + std::to_string(c) + " leaves the leaf");
    } else {
      const int l = 2 * c + 1, r = 2 * c + 2;
      cols = (so[l + 1] - so[l]) + (so[r + 1] - so[r]);
      // the children's skeletons lie in their ranges (checked first, going
      // bottom-up), so every index is a valid point id
      for (int64_t t = so[l]; t < so[r + 1]; ++t) stamp[pb->skel_index[t]] = c;
      for (int64_t t = so[c]; t < so[c + 1]; ++t) {
        const int32_t i = pb->skel_index[t];
        if (i < a || i >= b || stamp[i] != c)
          return fail_h(h, INVASKIT_E_ARG,
                        "skeleton of node " + std::to_string(c) +
                            " is not nested in its children's skeletons");
      }
    }
    if (po[c + 1] - po[c] != sc * cols)
      return fail_h(h, INVASKIT_E_ARG,
                    "P of node " + std::to_string(c) + " must have " + std::to_string(sc) + " x " +
                        std::to_string(cols) + " entries");
  }
  return INVASKIT_OK;
}

// ----------------------------------------------------------- table builders
// padded extent of N in the grouped GEMM's column tiles
int gemm_cols_padded(int n) {
  if (n <= kGemmMaxCols) return 16 * ((n + 15) / 16);
  return kGemmColChunk * ((n + kGemmColChunk - 1) / kGemmColChunk);
}
void gemm_tiles(std::vector<Tile3>& tiles, int prob, int M, int N) {
  const int ntn = N <= kGemmMaxCols ? 1 : (N + kGemmColChunk - 1) / kGemmColChunk;
  for (int tn = 0; tn < ntn; ++tn)
    for (int tm = 0; tm < (M + kGemmTileM - 1) / kGemmTileM; ++tm) tiles.push_back({prob, tm, tn});
}

struct GemmBuilder {
  std::vector<GemmProb> probs;
  std::vector<GemmSeg> segs;
  int begin(void* C, int64_t ldc, int M, int N, double alpha, double beta) {
    GemmProb p{};
    p.C = C;
    p.ldc = ldc;
    p.M = M;
    p.N = N;
    p.seg0 = (int)segs.size();
    p.nseg = 0;
    p.alpha = alpha;
    p.beta = beta;
    probs.push_back(p);
    return (int)probs.size() - 1;
  }
  void seg(const void* A, int64_t lda, bool a_rm, const void* B, int64_t ldb, int k) {
    if (k <= 0) return;
    GemmSeg g{};
    g.A = A;
    g.B = B;
    g.lda = lda;
    g.ldb = ldb;
    g.k = k;
    g.a_rm = a_rm ? 1 : 0;
    segs.push_back(g);
    probs.back().nseg++;
  }
  GemmL emit(Arena& ar) {
    // Skinny launches (every N <= kGemvCols) take a GEMV form, one workgroup
    // per product, when it pays (measured): column-major A with M <=
    // kGemvRows (the waves split K), or row-major A with long rows (mean K of
    // at least kGemvRmMinK: one wave per row).  Others take the tiles.
    {
      bool skinny = !probs.empty(), all_cm = true, all_rm = true;
      int mmax = 0;
      double ksum = 0.0;
      for (const GemmProb& p : probs) {
        skinny = skinny && p.N <= kGemvCols;
        mmax = std::max(mmax, p.M);
        for (int q = 0; q < p.nseg; ++q) {
          all_cm = all_cm && segs[p.seg0 + q].a_rm == 0;
          all_rm = all_rm && segs[p.seg0 + q].a_rm != 0;
          ksum += segs[p.seg0 + q].k;
        }
      }
      const bool cm_ok = all_cm && mmax <= kGemvRows;
      const bool rm_ok = all_rm && ksum >= (double)kGemvRmMinK * probs.size();
      if (skinny && all_cm && !cm_ok) {
        // tall: workgroups of kGemvTallRows rows, longest products first
        std::vector<int> order(probs.size());
        std::vector<double> kk(probs.size(), 0.0);
        for (size_t i = 0; i < probs.size(); ++i) {
          order[i] = (int)i;
          for (int q = 0; q < probs[i].nseg; ++q) kk[i] += segs[probs[i].seg0 + q].k;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return kk[x] > kk[y]; });
        std::vector<Tile3> tt;
        for (int i : order)
          for (int tm = 0; tm < (probs[i].M + kGemvTallRows - 1) / kGemvTallRows; ++tm)
            if (probs[i].N > 0) tt.push_back({i, tm, 0});
        GemmL l;
        l.gemv = kGemvTall;
        l.nprobs = (int)probs.size();
        l.probs = ar.add(probs);
        l.segs = ar.add(segs);
        l.tiles = ar.add(tt);
        l.ntiles = (int)tt.size();
        return l;
      }
      if (skinny && (cm_ok || rm_ok)) {
        GemmL l;
        l.gemv = cm_ok ? kGemvSplitK : kGemvRowMajor;
        l.nprobs = (int)probs.size();
        l.probs = ar.add(probs);
        l.segs = ar.add(segs);
        return l;
      }
    }
    // A product whose A operands are all row-major may be computed as
    // C^T = B^T A^T (B^T is then a row-major operand, A^T a column-major
    // one, and C^T is stored row-major, i.e. C column-major): chosen when
    // that needs fewer padded tile elements (few rows, many columns).
    std::vector<Tile3> tiles, tiles_t;
    std::vector<int64_t> cost(probs.size(), 0);
    std::vector<char> trans(probs.size(), 0);
    auto padded = [](int M, int N) {
      return (int64_t)((M + kGemmTileM - 1) / kGemmTileM) * kGemmTileM * gemm_cols_padded(N);
    };
    for (size_t i = 0; i < probs.size(); ++i) {
      GemmProb& p = probs[i];
      bool all_rm = p.nseg > 0;
      for (int q = 0; q < p.nseg; ++q) {
        cost[i] += segs[p.seg0 + q].k;
        all_rm = all_rm && segs[p.seg0 + q].a_rm;
      }
      if (p.M <= 0 || p.N <= 0) continue;
      if (all_rm && padded(p.N, p.M) < padded(p.M, p.N)) {
        for (int q = 0; q < p.nseg; ++q) {
          GemmSeg& g = segs[p.seg0 + q];
          std::swap(g.A, g.B);
          std::swap(g.lda, g.ldb);
          g.a_rm = 1;  // B (column-major K x N) read as the row-major N x K operand
        }
        std::swap(p.M, p.N);
        trans[i] = 1;
      }
    }
    // longest products first, so the launch does not end on a long tile; a
    // product's tiles stay consecutive (the products are sorted, stably, and
    // their tiles emitted in that order)
    std::vector<int> order(probs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return cost[x] > cost[y]; });
    for (int i : order) {
      const GemmProb& p = probs[i];
      if (p.M <= 0 || p.N <= 0) continue;
      gemm_tiles(trans[i] ? tiles_t : tiles, i, p.M, p.N);
    }
    GemmL l;
    l.probs = ar.add(probs);
    l.segs = ar.add(segs);
    l.tiles = ar.add(tiles);
    l.ntiles = (int)tiles.size();
    l.tiles_n = ar.add(tiles_t);
    l.ntiles_n = (int)tiles_t.size();
    return l;
  }
};

struct TrsmBuilder {
  std::vector<TrsmProb> probs;
  int nmax = 0;
  void add(const void* lu, const void* dinv, const int32_t* perm, int n, int nrhs, const void* in0,
           int64_t ld0, int split, const void* in1, int64_t ld1, void* out, int64_t ldo) {
    TrsmProb p{};
    p.lu = lu;
    p.dinv = dinv;
    p.perm = perm;
    p.n = n;
    p.nrhs = nrhs;
    p.in0 = in0;
    p.in1 = in1;
    p.ldin0 = ld0;
    p.ldin1 = ld1;
    p.split = split;
    p.out = out;
    p.ldout = ldo;
    probs.push_back(p);
    nmax = std::max(nmax, n);
  }
  TrsmL emit(Arena& ar, int tz64, int tv64, int kind, int cols = kTrsmColsDefault) {
    TrsmL l;
    if (getrs_lds_bytes(nmax, tz64 ? 8 : 4, cols) > (size_t)kLdsBytes) {
      l.ntiles = -1;  // the workgroup's right-hand sides do not fit in LDS
      return l;
    }
    // largest systems first (the systems are sorted, stably, and their
    // tiles emitted in that order, so a system's tiles stay consecutive)
    std::vector<int> order(probs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return probs[x].n > probs[y].n; });
    std::vector<Tile2> tiles;
    for (int i : order) {
      for (int tn = 0; tn < (probs[i].nrhs + cols - 1) / cols; ++tn) tiles.push_back({i, tn});
      l.work += (double)probs[i].n * probs[i].n * probs[i].nrhs;
    }
    l.probs = ar.add(probs);
    l.tiles = ar.add(tiles);
    l.ntiles = (int)tiles.size();
    l.nmax = nmax;
    l.tz64 = tz64;
    l.tv64 = tv64;
    l.kind = kind;
    l.cols = cols;
    return l;
  }
};


template <typename T>
T* offp(void* base, int64_t elems) {
  return static_cast<T*>(base) + elems;
}
inline void* offv(const void* base, int64_t elems, size_t esz) {
  return const_cast<unsigned char*>(static_cast<const unsigned char*>(base)) + elems * esz;
}

// ----------------------------------------------------------------- planning
// Tree-derived sizes and element offsets of every factor buffer (host only).
void layout_factor(H* h) {
  const int L = h->L;
  const int nn = h->nn;
  h->na.assign(nn, 0);
  h->nb.assign(nn, 0);
  h->s.assign(nn, 0);
  h->w.assign(nn, 0);
  h->z.assign(nn, 0);
  for (int c = 0; c < nn; ++c) {
    const int k = h->level(c);
    const int idx = c - ((1 << k) - 1);
    const int span = 1 << (L - k);
    h->na[c] = h->leaf_off[idx * span];
    h->nb[c] = h->leaf_off[(idx + 1) * span];
    h->s[c] = (int)(h->skel_off[c + 1] - h->skel_off[c]);
  }
  for (int c = 1; c < nn; ++c) h->w[c] = h->s[h->sib(c)];
  for (int c = 0; c < nn; ++c)
    if (!h->is_leaf(c)) h->z[c] = h->s[2 * c + 1] + h->s[2 * c + 2];

  // Sweep columns of every node: factor levels k = level(c) .. 1, each
  // w_{anc_k(c)} wide, in that order (a leaf's are its W storage columns).
  h->colp.assign(nn, std::vector<int>());
  h->Ssw.assign(nn, 0);
  for (int c = 1; c < nn; ++c) {
    const int lev = h->level(c);
    h->colp[c].assign(lev + 1, 0);
    int run = 0;
    for (int k = lev; k >= 1; --k) {
      h->colp[c][k] = run;
      run += h->w[h->anc(c, k)];
    }
    h->Ssw[c] = run;
  }
  // leaf LU and leaf-major W storage (m x Ssw[leaf], column-major)
  h->lu_off.assign(h->nleaves + 1, 0);
  h->slab_off.assign(h->nleaves + 1, 0);
  h->S.assign(h->nleaves, 0);
  h->colk.assign(h->nleaves, std::vector<int>(L + 1, 0));
  for (int j = 0; j < h->nleaves; ++j) {
    const int lf = h->leaf_node(j);
    const int64_t m = h->nb[lf] - h->na[lf];
    h->lu_off[j + 1] = h->lu_off[j] + m * m;
    for (int k = L; k >= 1; --k) h->colk[j][k] = h->colp[lf][k];
    h->S[j] = L > 0 ? h->Ssw[lf] : 0;
    h->slab_off[j + 1] = h->slab_off[j] + m * h->S[j];
  }
  // reduced systems
  h->zis64.assign(L + 1, 1);
  if (h->prec == INVASKIT_PREC_MIXED)
    for (int k = 0; k <= L; ++k) h->zis64[k] = (k < h->top64) ? 1 : 0;
  h->z_off.assign(nn, 0);
  h->zperm_off.assign(nn + 1, 0);
  int64_t z64n = 0, zTn = 0, zpn = 0;
  const int ninternal = (1 << L) - 1;
  for (int c = 0; c < ninternal; ++c) {
    const int64_t zz = (int64_t)h->z[c] * h->z[c];
    if (h->zis64[h->level(c)]) {
      h->z_off[c] = z64n;
      z64n += zz;
    } else {
      h->z_off[c] = zTn;
      zTn += zz;
    }
    h->zperm_off[c] = zpn;
    zpn += h->z[c];
  }
  // inverses of the 64 x 64 diagonal blocks of every LU factor
  auto nblk = [](int64_t m) { return (m + kDiagBlock - 1) / kDiagBlock; };
  constexpr int64_t kDB2 = 2 * kDiagBlock * kDiagBlock;
  h->dleaf_off.assign(h->nleaves + 1, 0);
  for (int j = 0; j < h->nleaves; ++j) {
    const int lf = h->leaf_node(j);
    h->dleaf_off[j + 1] = h->dleaf_off[j] + nblk(h->nb[lf] - h->na[lf]) * kDB2;
  }
  h->dz_off.assign(nn, 0);
  int64_t dz64 = 0, dzT = 0;
  for (int c = 0; c < ninternal; ++c) {
    const int64_t e = nblk(h->z[c]) * kDB2;
    if (h->zis64[h->level(c)]) {
      h->dz_off[c] = dz64;
      dz64 += e;
    } else {
      h->dz_off[c] = dzT;
      dzT += e;
    }
  }
  // skeleton projections (every non-root node) and sweep solutions (internal
  // nodes below the root) for all factor levels at once
  h->psw_off.assign(nn, 0);
  h->ysw_off.assign(nn, 0);
  int64_t pn = 0, yn = 0;
  for (int c = 1; c < nn; ++c) {
    h->psw_off[c] = pn;
    pn += (int64_t)h->s[c] * h->Ssw[c];
    if (!h->is_leaf(c)) {
      h->ysw_off[c] = yn;
      yn += (int64_t)h->z[c] * h->Ssw[c];
    }
  }
  h->z64n = z64n;
  h->zTn = zTn;
  h->zpn = zpn;
  h->dz64n = dz64;
  h->dzTn = dzT;
  h->pswn = pn;
  h->yswn = yn;
}

// Carves the handle's buffers from the region at `base` (kPlanBase when only
// sizes are wanted); the descriptor tables come last, table_bytes long.
// Plain handles keep their own device copies of the skeleton indices and (in
// mixed precision) of P in FP32; a sweep's handles use the sweep's
// (shared != nullptr).  Returns the region's size.
size_t carve_factor(H* h, unsigned char* base, const KernelCache* shared, size_t table_bytes) {
  Carve cv;
  const size_t es = h->tsize();
  auto put = [&](Buf& b, size_t bytes) {
    const size_t o = cv.take(bytes);
    b.p = base + o;
    b.bytes = bytes;
  };
  const int ninternal = (1 << h->L) - 1;
  // factor storage is padded by one 64-column block: the solves read factor
  // rows as whole vectors past the last partial block
  put(h->leafLU, (h->lu_off[h->nleaves] + kDiagBlock) * es);
  put(h->leafPerm, sizeof(int32_t) * h->N);
  put(h->leafInfo, sizeof(int32_t) * h->nleaves);
  put(h->slab, std::max<int64_t>(h->slab_off[h->nleaves], 1) * es);
  put(h->Z64, (h->z64n + kDiagBlock) * 8);
  put(h->ZT, (h->zTn + kDiagBlock) * es);
  put(h->zperm, sizeof(int32_t) * std::max<int64_t>(h->zpn, 1));
  put(h->zinfo, sizeof(int32_t) * std::max(ninternal, 1));
  put(h->dinvLeaf, h->dleaf_off[h->nleaves] * es);
  put(h->dinvZ64, std::max<int64_t>(h->dz64n, 1) * 8);
  put(h->dinvZT, std::max<int64_t>(h->dzTn, 1) * es);
  put(h->psw, std::max<int64_t>(h->pswn, 1) * es);
  put(h->ysw, std::max<int64_t>(h->yswn, 1) * es);
  const bool mixed = h->prec == INVASKIT_PREC_MIXED;
  if (!shared) {
    put(h->skel_own, sizeof(int32_t) * std::max<size_t>(h->skel_idx.size(), 1));
    if (mixed) put(h->P32_own, sizeof(float) * std::max<int64_t>(h->p_off[h->nn], 1));
    h->skd = static_cast<const int32_t*>(h->skel_own.p);
    h->Pf = mixed ? h->P32_own.p : static_cast<const void*>(h->P64);
  } else {
    h->skd = static_cast<const int32_t*>(shared->skel.p);
    h->Pf = mixed ? shared->P32.p : static_cast<const void*>(h->P64);
  }
  put(h->fp.tables, table_bytes);
  h->region = base;
  h->region_bytes = cv.total();
  return h->region_bytes;
}

// The shared part of a sweep's workspace: lambda-free kernel blocks in the
// factor storage layout, skeleton indices and FP32 P.
size_t carve_cache(const H* h, KernelCache& kc, unsigned char* base) {
  Carve cv;
  const size_t es = h->tsize();
  auto put = [&](Buf& b, size_t bytes) {
    const size_t o = cv.take(bytes);
    b.p = base + o;
    b.bytes = bytes;
  };
  put(kc.leaf, h->lu_off[h->nleaves] * es);
  put(kc.slab, std::max<int64_t>(h->slab_off[h->nleaves], 1) * es);
  put(kc.skel, sizeof(int32_t) * std::max<size_t>(h->skel_idx.size(), 1));
  if (h->prec == INVASKIT_PREC_MIXED)
    put(kc.P32, sizeof(float) * std::max<int64_t>(h->p_off[h->nn], 1));
  return cv.total();
}

// Descriptor tables of the factorization of the handles `hs` (identical
// layouts; several handles: the lambdas of a sweep batched into the same
// launches).  kc != nullptr: the kernel blocks are evaluated once into the
// cache and read from it (leaf blocks copied with each handle's lambda on
// the diagonal; the leaf solves read the skeleton blocks from the cache and
// write each handle's W storage).
void build_factor_tables(const std::vector<H*>& hs, const KernelCache* kc, Arena& ar,
                         FactorPlan& fp) {
  H* h = hs[0];
  const int L = h->L;
  const size_t es = h->tsize();
  const int T64 = (h->prec == INVASKIT_PREC_FP64) ? 1 : 0;
  const Buf tables = fp.tables;
  fp = FactorPlan();
  fp.tables = tables;
  fp.cached = kc != nullptr;
  constexpr int64_t kDB2 = 2 * kDiagBlock * kDiagBlock;
  const int32_t* skd = h->skd;
  // leaf blocks and their LU; skeleton blocks, leaf solves and leaf
  // projections of every level
  {
    std::vector<EvalBlock> lblocks, pblocks;
    std::vector<Tile3> ltiles, ptiles;
    std::vector<CopyShiftProb> copies;
    std::vector<LuProb> lus[2];
    std::vector<DiagInvProb> dis[2];
    TrsmBuilder tb[2];
    GemmBuilder proj[2];
    int nmax[2] = {0, 0};
    const int small_leaf = T64 ? kSmallLeaf64 : kSmallLeaf32;
    for (size_t g = 0; g < hs.size(); ++g) {
      H* hg = hs[g];
      for (int j = 0; j < h->nleaves; ++j) {
        const int lf = h->leaf_node(j);
        const int m = (int)(h->nb[lf] - h->na[lf]);
        void* lu = offv(hg->leafLU.p, h->lu_off[j], es);
        if (g == 0) {
          EvalBlock b{};
          b.out = kc ? offv(kc->leaf.p, h->lu_off[j], es) : lu;
          b.ld = m;
          b.row0 = h->na[lf];
          b.cols = nullptr;
          b.col0 = h->na[lf];
          b.rows = m;
          b.ncols = m;
          b.diag = 1;
          lblocks.push_back(b);
          for (int tn = 0; tn < (m + kEvalTile - 1) / kEvalTile; ++tn)
            for (int tm = 0; tm < (m + kEvalTile - 1) / kEvalTile; ++tm)
              ltiles.push_back({(int)lblocks.size() - 1, tm, tn});
        }
        if (kc) {
          CopyShiftProb c{};
          c.src = offv(kc->leaf.p, h->lu_off[j], es);
          c.dst = lu;
          c.m = m;
          c.shift = hg->lam;
          copies.push_back(c);
        }
        const int cls = m <= small_leaf ? 1 : 0;
        LuProb p{};
        p.a = lu;
        p.perm = static_cast<int32_t*>(hg->leafPerm.p) + h->na[lf];
        p.info = static_cast<int32_t*>(hg->leafInfo.p) + j;
        p.n = m;
        lus[cls].push_back(p);
        nmax[cls] = std::max(nmax[cls], m);
        fp.leaf_lu[cls].work += (double)m * m * m;
        for (int jb = 0; jb < m; jb += kDiagBlock) {
          DiagInvProb d{};
          d.lu = lu;
          d.perm = p.perm;
          d.out = offv(hg->dinvLeaf.p, h->dleaf_off[j] + (jb / kDiagBlock) * kDB2, es);
          d.n = m;
          d.jb = jb;
          dis[cls].push_back(d);
        }
        if (L == 0) continue;
        void* slab = offv(hg->slab.p, h->slab_off[j], es);
        void* kin = kc ? offv(kc->slab.p, h->slab_off[j], es) : slab;
        if (g == 0) {
          for (int k = L; k >= 1; --k) {
            const int c = h->anc(lf, k);
            const int wk = h->w[c];
            EvalBlock e{};
            e.out = offv(kin, (int64_t)h->colk[j][k] * m, es);
            e.ld = m;
            e.row0 = h->na[lf];
            e.cols = skd + h->skel_off[h->sib(c)];
            e.rows = m;
            e.ncols = wk;
            e.diag = 0;
            pblocks.push_back(e);
            for (int tn = 0; tn < (wk + kEvalTile - 1) / kEvalTile; ++tn)
              for (int tm = 0; tm < (m + kEvalTile - 1) / kEvalTile; ++tm)
                ptiles.push_back({(int)pblocks.size() - 1, tm, tn});
          }
        }
        tb[cls].add(lu, hg->DL(j), static_cast<const int32_t*>(hg->leafPerm.p) + h->na[lf], m,
                    h->S[j], kin, m, m, kin, m, slab, m);
        proj[cls].begin(offv(hg->psw.p, h->psw_off[lf], es), h->s[lf], h->s[lf], h->S[j], 1.0,
                        0.0);
        proj[cls].seg(offv(hg->Pt(), h->p_off[lf], es), m, true, slab, m, m);
      }
    }
    fp.leaf_eval.blocks = ar.add(lblocks);
    fp.leaf_eval.tiles = ar.add(ltiles);
    fp.leaf_eval.ntiles = (int)ltiles.size();
    fp.leaf_eval.nblocks = (int)lblocks.size();
    fp.leaf_copy.probs = ar.add(copies);
    fp.leaf_copy.count = (int)copies.size();
    // largest matrices first: one workgroup per matrix, so the launch's tail
    // is set by the matrices dispatched last
    auto by_order = [](const LuProb& x, const LuProb& y) { return x.n > y.n; };
    for (int c = 0; c < 2; ++c) {
      std::stable_sort(lus[c].begin(), lus[c].end(), by_order);
      fp.leaf_lu[c].probs = ar.add(lus[c]);
      fp.leaf_lu[c].count = (int)lus[c].size();
      fp.leaf_lu[c].nmax = nmax[c];
      fp.leaf_lu[c].t64 = T64;
      fp.leaf_dinv[c].probs = ar.add(dis[c]);
      fp.leaf_dinv[c].count = (int)dis[c].size();
      fp.leaf_dinv[c].t64 = T64;
    }
    fp.panels.blocks = ar.add(pblocks);
    fp.panels.tiles = ar.add(ptiles);
    fp.panels.ntiles = (int)ptiles.size();
    fp.panels.nblocks = (int)pblocks.size();
    for (int c = 0; c < 2; ++c) {
      fp.leaf_trsm[c][0] = tb[c].emit(ar, T64, T64, 0, 16);
      fp.leaf_trsm[c][1] = tb[c].emit(ar, T64, T64, 0, 32);
    }
    for (int c = 0; c < 2; ++c) fp.leaf_proj[c] = proj[c].emit(ar);
  }
  // wavefront over levels j = L-1 .. 0
  fp.zform.assign(std::max(L, 1), ZformL());
  fp.zlu.assign(std::max(L, 1), LuL());
  fp.zdinv.assign(std::max(L, 1), DinvL());
  fp.zsolve.assign(std::max(L, 1), TrsmL());
  fp.zsolve32.assign(std::max(L, 1), TrsmL());
  fp.pgemm.assign(std::max(L, 1), GemmL());
  for (int jl = L - 1; jl >= 0; --jl) {
    std::vector<ZformProb> zf;
    std::vector<LuProb> zl;
    std::vector<DiagInvProb> zd;
    TrsmBuilder zs;
    GemmBuilder pg;
    int nmax = 0;
    const size_t zes = h->zis64[jl] ? 8 : es;
    for (size_t g = 0; g < hs.size(); ++g) {
      H* hg = hs[g];
      int32_t* zpm = static_cast<int32_t*>(hg->zperm.p);
      void* PS = hg->psw.p;
      void* YS = hg->ysw.p;
      const void* Pt = hg->Pt();
      for (int a = (1 << jl) - 1; a < (2 << jl) - 1; ++a) {
        for (int jb = 0; jb < h->z[a]; jb += kDiagBlock) {
          DiagInvProb d{};
          d.lu = hg->Z(a);
          d.perm = zpm + h->zperm_off[a];
          d.out = offv(hg->DZ(a), (jb / kDiagBlock) * kDB2, zes);
          d.n = h->z[a];
          d.jb = jb;
          zd.push_back(d);
        }
        const int l = 2 * a + 1, r = 2 * a + 2;
        ZformProb p{};
        p.Z = hg->Zm(a);
        p.pr = offv(PS, h->psw_off[r], es);  // first columns: factor level jl+1
        p.pl = offv(PS, h->psw_off[l], es);
        p.sr = h->s[r];
        p.sl = h->s[l];
        zf.push_back(p);
        LuProb q{};
        q.a = hg->Zm(a);
        q.perm = zpm + h->zperm_off[a];
        q.info = static_cast<int32_t*>(hg->zinfo.p) + a;
        q.n = h->z[a];
        zl.push_back(q);
        nmax = std::max(nmax, h->z[a]);
        if (jl >= 1) {
          void* y = offv(YS, h->ysw_off[a], es);
          zs.add(hg->Z(a), hg->DZ(a), zpm + h->zperm_off[a], h->z[a], h->Ssw[a],
                 offv(PS, h->psw_off[r] + (int64_t)h->colp[r][jl] * h->s[r], es), h->s[r],
                 h->s[r], offv(PS, h->psw_off[l] + (int64_t)h->colp[l][jl] * h->s[l], es),
                 h->s[l], y, h->z[a]);
          pg.begin(offv(PS, h->psw_off[a], es), h->s[a], h->s[a], h->Ssw[a], 1.0, 0.0);
          const void* Pa = offv(Pt, h->p_off[a], es);
          pg.seg(Pa, h->z[a], true, offv(y, h->s[r], es), h->z[a], h->s[l]);
          pg.seg(offv(Pa, h->s[l], es), h->z[a], true, y, h->z[a], h->s[r]);
        }
      }
    }
    ZformL& zfl = fp.zform[jl];
    zfl.probs = ar.add(zf);
    zfl.count = (int)zf.size();
    zfl.tz64 = h->zis64[jl];
    zfl.tv64 = T64;
    LuL& lul = fp.zlu[jl];
    std::stable_sort(zl.begin(), zl.end(), [](const LuProb& x, const LuProb& y) { return x.n > y.n; });
    lul.probs = ar.add(zl);
    lul.count = (int)zl.size();
    lul.nmax = nmax;
    lul.t64 = h->zis64[jl];
    lul.kind = 1;
    DinvL& dl = fp.zdinv[jl];
    dl.probs = ar.add(zd);
    dl.count = (int)zd.size();
    dl.t64 = h->zis64[jl];
    if (jl >= 1) {
      fp.zsolve[jl] = zs.emit(ar, h->zis64[jl], T64, 1);
      fp.zsolve32[jl] = zs.emit(ar, h->zis64[jl], T64, 1, 32);
      fp.pgemm[jl] = pg.emit(ar);
    }
  }
}

// Size of one handle's factor tables (a placeholder-base planning run).
size_t factor_table_bytes(H* h, const KernelCache* kc) {
  Arena ar;
  FactorPlan fp;
  build_factor_tables({h}, kc, ar, fp);
  return ar.bytes();
}

// ---------------------------------------------------------------- launching
hipError_t run_gemm(const Buf& tb, const GemmL& l, bool f64, hipStream_t s) {
  const GemmProb* p = at<GemmProb>(tb, l.probs);
  const GemmSeg* g = at<GemmSeg>(tb, l.segs);
  if (l.gemv == kGemvTall)
    return f64 ? launch_gemv_tall<double>(p, g, at<Tile3>(tb, l.tiles), l.ntiles, s)
               : launch_gemv_tall<float>(p, g, at<Tile3>(tb, l.tiles), l.ntiles, s);
  if (l.gemv)
    return f64 ? launch_gemv<double>(p, g, l.nprobs, l.gemv, s)
               : launch_gemv<float>(p, g, l.nprobs, l.gemv, s);
  hipError_t e = hipSuccess;
  if (l.ntiles > 0)
    e = f64 ? launch_gemm<double>(p, g, at<Tile3>(tb, l.tiles), l.ntiles, false, s)
            : launch_gemm<float>(p, g, at<Tile3>(tb, l.tiles), l.ntiles, false, s);
  if (e == hipSuccess && l.ntiles_n > 0)
    e = f64 ? launch_gemm<double>(p, g, at<Tile3>(tb, l.tiles_n), l.ntiles_n, true, s)
            : launch_gemm<float>(p, g, at<Tile3>(tb, l.tiles_n), l.ntiles_n, true, s);
  return e;
}

hipError_t run_trsm(const Buf& tb, const TrsmL& l, hipStream_t s) {
  if (l.ntiles == 0) return hipSuccess;
  if (l.ntiles < 0) return hipErrorInvalidValue;
  const TrsmProb* p = at<TrsmProb>(tb, l.probs);
  const Tile2* t = at<Tile2>(tb, l.tiles);
  if (l.tz64 && l.tv64)
    return launch_getrs<double, double>(p, t, l.ntiles, l.nmax, l.kind, l.cols, s);
  if (l.tz64) return launch_getrs<double, float>(p, t, l.ntiles, l.nmax, l.kind, l.cols, s);
  return launch_getrs<float, float>(p, t, l.ntiles, l.nmax, l.kind, l.cols, s);
}

hipError_t run_lu(const Buf& tb, const LuL& l, hipStream_t s) {
  if (l.count == 0) return hipSuccess;
  if (l.t64)
    return launch_getrf<double>(at<LuProb>(tb, l.probs), l.count, l.nmax, l.kind, l.panel,
                                l.waves, s, l.form, l.nopiv);
  return launch_getrf<float>(at<LuProb>(tb, l.probs), l.count, l.nmax, l.kind, l.panel, l.waves,
                             s, l.form, l.nopiv);
}

hipError_t run_dinv(const Buf& tb, const DinvL& l, hipStream_t s) {
  if (l.count == 0) return hipSuccess;
  if (l.t64) return launch_diag_inv<double>(at<DiagInvProb>(tb, l.probs), l.count, s);
  return launch_diag_inv<float>(at<DiagInvProb>(tb, l.probs), l.count, s);
}

hipError_t run_zform(const Buf& tb, const ZformL& l, hipStream_t s) {
  if (l.count == 0) return hipSuccess;
  const ZformProb* p = at<ZformProb>(tb, l.probs);
  if (l.tz64 && l.tv64) return launch_zform<double, double>(p, l.count, s);
  if (l.tz64) return launch_zform<double, float>(p, l.count, s);
  return launch_zform<float, float>(p, l.count, s);
}

hipError_t run_eval(H* h, const Buf& tb, const EvalL& l, double shift, hipStream_t s) {
  if (l.ntiles == 0) return hipSuccess;
  const EvalBlock* b = at<EvalBlock>(tb, l.blocks);
  const Tile3* t = at<Tile3>(tb, l.tiles);
  const bool f64 = h->prec == INVASKIT_PREC_FP64;
  if (h->pdt == INVASKIT_F64) {
    const double* X = static_cast<const double*>(h->X);
    return f64 ? launch_eval<double, double>(X, h->d, h->h, shift, b, t, l.ntiles, s)
               : launch_eval<double, float>(X, h->d, h->h, shift, b, t, l.ntiles, s);
  }
  const float* X = static_cast<const float*>(h->X);
  return f64 ? launch_eval<float, double>(X, h->d, h->h, shift, b, t, l.ntiles, s)
             : launch_eval<float, float>(X, h->d, h->h, shift, b, t, l.ntiles, s);
}

hipError_t run_copy_shift(H* h, const Buf& tb, const CopyShiftL& l, hipStream_t s) {
  if (l.count == 0) return hipSuccess;
  const CopyShiftProb* p = at<CopyShiftProb>(tb, l.probs);
  return h->prec == INVASKIT_PREC_FP64 ? launch_copy_shift<double>(p, l.count, s)
                                       : launch_copy_shift<float>(p, l.count, s);
}

// ---------------------------------------------------------------- autotuning
// Process-wide table: shape class of a launch -> chosen tile parameter.
struct TuneTable {
  std::mutex mu;
  std::map<std::string, int> choice;
};
TuneTable& tune_table() {
  static TuneTable t;
  return t;
}

// half-octave bin of a positive count
int tune_bin(double x) { return x > 0 ? (int)std::lround(2.0 * std::log2(x)) : -1; }

std::string lu_key(const LuL& l) {
  return std::string("getrf.") + (l.t64 ? "f64" : "f32") + (l.nopiv ? ".np" : "") + ".n" +
         std::to_string(l.nmax) + ".c" + std::to_string(tune_bin(l.count)) + ".w" +
         std::to_string(tune_bin(l.work));
}
std::string trsm_key(const TrsmL& l) {
  return std::string("getrs.") + (l.tz64 ? "f64" : "f32") + ".k" + std::to_string(l.kind) +
         ".n" + std::to_string(l.nmax) + ".w" + std::to_string(tune_bin(l.work));
}
std::string zlu_key(const LuL& l) {
  return std::string("zgetrf.") + (l.t64 ? "f64" : "f32") + ".n" + std::to_string(l.nmax) +
         ".c" + std::to_string(tune_bin(l.count));
}

// Best of two timed runs of `launch` on stream s, each after `prepare`
// (events e0 and e1 are the caller's).
template <typename Prep, typename Launch>
hipError_t best_of_two(hipStream_t s, hipEvent_t e0, hipEvent_t e1, Prep&& prepare,
                       Launch&& launch, float& best) {
  best = 0.f;
  hipError_t e = hipSuccess;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
    e = prepare();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (best == 0.f || ms < best)) best = ms;
  }
  return e;
}

// The level wavefront's choices at level j: the LU form of the reduced
// systems and the sweep solves' right-hand sides per workgroup, fixed by the
// options, found in the table, or timed here, on stream s, before the
// level's own launches.  Rebuilding Z from the children's projections makes
// every LU trial start from the same matrices; the solves read the
// projections and write Y only, so their trials change nothing else.
int tune_level(H* h, const Buf& tb, const FactorPlan& fp, int j, hipStream_t s, int* form,
               int* cols) {
  const LuL& zl = fp.zlu[j];
  const bool can_one = zl.count > 0 && zl.nmax <= kOneWaveMax;
  const bool has_solve = j >= 1 && fp.zsolve[j].ntiles > 0;
  const bool can32 = has_solve && fp.zsolve32[j].ntiles >= 0;
  int f = can_one ? h->fix_zlu_form : kLuFormBlock;
  int c = has_solve ? h->fix_zsolve_cols : kTrsmColsDefault;
  if (c == 32 && !can32)
    return fail_h(h, INVASKIT_E_ARG,
                  "zsolve_cols = 32 needs more than 160 KiB of LDS at this reduced-system size");
  if (!c && !can32) c = kTrsmColsDefault;
  if (h->tune == INVASKIT_TUNE_OFF) {
    if (!f) f = zl.t64 ? kLuFormBlock : kLuFormOneWave;
    if (!c) c = kTrsmColsDefault;
  }
  const std::string kz = zlu_key(zl), ks = has_solve ? trsm_key(fp.zsolve[j]) : std::string();
  {
    std::lock_guard<std::mutex> g(tune_table().mu);
    auto& t = tune_table().choice;
    if (!f && t.count(kz)) f = t[kz];
    if (!c && t.count(ks)) c = t[ks];
  }
  if (!f || !c) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      hipEventDestroy(e0);
      return fail_h(h, INVASKIT_E_HIP, "hipEventCreate failed");
    }
    hipError_t e = hipSuccess;
    auto lu_form = [&](int form_) {
      LuL l = zl;
      l.form = form_;
      return run_lu(tb, l, s);
    };
    auto zform = [&]() { return run_zform(tb, fp.zform[j], s); };
    const bool tuned_f = !f, tuned_c = !c;
    if (!f) {
      float t1 = 0.f, t2 = 0.f;
      e = best_of_two(s, e0, e1, zform, [&]() { return lu_form(kLuFormOneWave); }, t1);
      if (e == hipSuccess)
        e = best_of_two(s, e0, e1, zform, [&]() { return lu_form(kLuFormBlock); }, t2);
      f = t1 <= t2 ? kLuFormOneWave : kLuFormBlock;
    }
    if (!c && e == hipSuccess) {
      // the solves read the level's factors and their diagonal-block inverses
      e = zform();
      if (e == hipSuccess) e = lu_form(f);
      if (e == hipSuccess) e = run_dinv(tb, fp.zdinv[j], s);
      float t16 = 0.f, t32 = 0.f;
      auto none = []() { return hipSuccess; };
      if (e == hipSuccess)
        e = best_of_two(s, e0, e1, none, [&]() { return run_trsm(tb, fp.zsolve[j], s); }, t16);
      if (e == hipSuccess)
        e = best_of_two(s, e0, e1, none, [&]() { return run_trsm(tb, fp.zsolve32[j], s); }, t32);
      c = t32 < t16 ? 32 : 16;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess)
      return fail_h(h, INVASKIT_E_HIP, std::string("level tuning: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> g(tune_table().mu);
    auto& t = tune_table().choice;
    if (tuned_f) t[kz] = f;
    if (tuned_c) t[ks] = c;
  }
  *form = f;
  *cols = c;
  return INVASKIT_OK;
}

// Settles the leaf LU's panel width and waves per matrix and the leaf
// solves' right-hand sides per workgroup for this factor: fixed by the
// options, found in the table, or timed.  A trial re-evaluates its launch's
// inputs first (both launches work in place) and is timed by events on the
// factor's stream; each candidate runs twice and keeps its faster time.  The
// trials leave the factor buffers in an arbitrary state: the factorization
// that follows rebuilds them.
int tune_factor(H* h, const FactorPlan& fp) {
  const Buf& tb = fp.tables;
  const bool f64 = h->prec == INVASKIT_PREC_FP64;
  hipStream_t s = h->stream;
  invaskit_tile_config& tc = h->tiles;
  tc = invaskit_tile_config{};
  // the LU tiles are timed on the class that runs the block kernel: the
  // large leaves, or the small ones when there are no large ones
  const int luc = fp.leaf_lu[0].count > 0 ? 0 : 1;
  LuL LU = fp.leaf_lu[luc];
  LU.nopiv = h->leaf_nopiv;
  const bool lu_choice = LU.count > 0 && (LU.t64 || LU.nmax > kSmallLeaf32);
  const std::string klu = lu_key(LU), klw = "getrfw" + klu.substr(5);
  bool has32[2], has_trsm[2];
  std::string ktr[2];
  int tr[2];
  for (int c = 0; c < 2; ++c) {
    has32[c] = fp.leaf_trsm[c][1].ntiles >= 0;
    has_trsm[c] = h->L > 0 && fp.leaf_trsm[c][0].ntiles > 0;
    ktr[c] = trsm_key(fp.leaf_trsm[c][0]);
    tr[c] = h->fix_trsm_cols;
    if (tr[c] == 32 && has_trsm[c] && !has32[c])
      return fail_h(h, INVASKIT_E_ARG,
                    "leaf_trsm_cols = 32 needs more than 160 KiB of LDS at this leaf size");
    if (!tr[c] && (!has32[c] || !has_trsm[c])) tr[c] = kTrsmColsDefault;
  }
  int lu = h->fix_lu_panel, lw = h->fix_lu_waves;
  if (f64 && h->fix_lu_panel == 32 && h->fix_lu_waves == 8)
    return fail_h(h, INVASKIT_E_ARG, "the FP64 leaf LU has no panel 32 at 8 waves");
  if (!lu && !lu_choice) lu = getrf_default_panel(f64);
  if (!lw && !lu_choice) lw = 4;
  if (h->tune == INVASKIT_TUNE_OFF) {
    if (!lu) lu = getrf_default_panel(f64);
    if (!lw) lw = 4;
    for (int& t : tr)
      if (!t) t = kTrsmColsDefault;
  }
  {
    std::lock_guard<std::mutex> g(tune_table().mu);
    auto& t = tune_table().choice;
    // a shape class's LU entry stands only as a pair (panel, waves)
    if (!lu && !lw && t.count(klu) && t.count(klw)) {
      lu = t[klu];
      lw = t[klw];
    }
    for (int c = 0; c < 2; ++c)
      if (!tr[c] && t.count(ktr[c])) tr[c] = t[ktr[c]];
  }
  if (!lu || !lw || !tr[0] || !tr[1]) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      hipEventDestroy(e0);
      return fail_h(h, INVASKIT_E_HIP, "hipEventCreate failed");
    }
    hipError_t e = hipSuccess;
    // best of two runs of `launch`, each after `prepare`
    auto trial = [&](auto&& prepare, auto&& launch, float& best) {
      best = 0.f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = prepare();
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (best == 0.f || ms < best)) best = ms;
      }
    };
    // the LU works in place: every trial starts from fresh leaf blocks (a
    // cached plan copies them from the evaluated cache)
    auto eval_leaves = [&]() {
      return fp.cached ? run_copy_shift(h, tb, fp.leaf_copy, s)
                       : run_eval(h, tb, fp.leaf_eval, h->lam, s);
    };
    auto lu_with = [&](const LuL& base, int panel, int waves) {
      LuL l = base;
      l.panel = panel;
      l.waves = waves;
      l.nopiv = h->leaf_nopiv;
      return run_lu(tb, l, s);
    };
    if (!lu || !lw) {
      // candidates (panel, waves) in the order of lu_ms; a fixed one of the
      // two restricts the others
      const int cp[4] = {16, 32, 16, 32}, cw[4] = {4, 4, 8, 8};
      float best = 0.f;
      int bi = -1;
      for (int i = 0; i < 4 && e == hipSuccess; ++i) {
        if ((lu && cp[i] != lu) || (lw && cw[i] != lw)) continue;
        if (f64 && cp[i] == 32 && cw[i] == 8) continue;  // not built
        trial(eval_leaves, [&]() { return lu_with(LU, cp[i], cw[i]); }, tc.lu_ms[i]);
        if (e == hipSuccess && (bi < 0 || tc.lu_ms[i] < best)) {
          best = tc.lu_ms[i];
          bi = i;
        }
      }
      if (bi >= 0) {
        lu = cp[bi];
        lw = cw[bi];
      }
    }
    if ((!tr[0] || !tr[1]) && e == hipSuccess) {
      // the solves need the leaf factors and their diagonal-block inverses
      e = eval_leaves();
      for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        e = lu_with(fp.leaf_lu[c], lu, lw);
        if (e == hipSuccess) e = run_dinv(tb, fp.leaf_dinv[c], s);
      }
      // in place unless the solves read the cache
      auto eval_panels = [&]() {
        return fp.cached ? hipSuccess : run_eval(h, tb, fp.panels, 0.0, s);
      };
      for (int c = 0; c < 2; ++c) {
        if (tr[c]) continue;
        float* ms = c == 0 ? tc.trsm_ms : tc.trsm_small_ms;
        trial(eval_panels, [&]() { return run_trsm(tb, fp.leaf_trsm[c][0], s); }, ms[0]);
        trial(eval_panels, [&]() { return run_trsm(tb, fp.leaf_trsm[c][1], s); }, ms[1]);
        tr[c] = ms[1] < ms[0] ? 32 : 16;
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess)
      return fail_h(h, INVASKIT_E_HIP, std::string("tile tuning: ") + hipGetErrorString(e));
    tc.tuned = 1;
    std::lock_guard<std::mutex> g(tune_table().mu);
    auto& t = tune_table().choice;
    if (!h->fix_lu_panel && !h->fix_lu_waves && lu_choice) {
      t[klu] = lu;
      t[klw] = lw;
    }
    for (int c = 0; c < 2; ++c)
      if (!h->fix_trsm_cols && has32[c] && has_trsm[c]) t[ktr[c]] = tr[c];
  }
  tc.leaf_lu_panel = lu;
  tc.leaf_lu_waves = lw;
  tc.leaf_trsm_cols = tr[0];
  tc.leaf_trsm_cols_small = fp.leaf_lu[1].count > 0 ? tr[1] : 0;
  return INVASKIT_OK;
}

// Runs the factorization plan `fp` over the handles `hs` (hs[0] leads: its
// stream, second stream, events and tile choices serve the launches).  A
// cached plan first makes sure the sweep's lambda-free kernel blocks are
// evaluated.  Phase times are recorded in every member.
int run_factor_once(const std::vector<H*>& hs, const FactorPlan& fp, KernelCache* kc,
                    bool* repivot) {
  H* h = hs[0];
  hipStream_t s = h->stream;
  const bool f64 = h->prec == INVASKIT_PREC_FP64;
  const Buf& tb = fp.tables;
  if (!h->have_events) {
    for (auto& e : h->ev) HIP_TRY(h, hipEventCreate(&e));
    h->have_events = true;
  }
  if (!h->side) HIP_TRY(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  hipStream_t s2 = h->side;
  // the members' pivot status (leaf blocks, reduced systems) is read back
  // into the pinned buffer with the factorization
  std::vector<size_t> info_at(hs.size() + 1, 0);
  for (size_t g = 0; g < hs.size(); ++g)
    info_at[g + 1] = info_at[g] + hs[g]->nleaves + std::max((1 << hs[g]->L) - 1, 0);
  int32_t* info_host = nullptr;
  {
    void* p = nullptr;
    if (int rc = host_pinned(h, sizeof(int32_t) * info_at.back(), &p)) return rc;
    info_host = static_cast<int32_t*>(p);
  }
  // Phase timing: each phase is bracketed by two events on the stream it
  // runs on; phases on the two streams overlap, so they need not sum to the
  // total.  `join` events order the streams.
  struct Bracket {
    hipEvent_t a, b;
    int phase;
  };
  std::vector<Bracket> brackets;
  int open_on[2] = {-1, -1};
  size_t used[2] = {0, 0};  // events of h->fev taken by this factorization
  auto new_event = [&](unsigned flags) -> hipEvent_t {
    const int k = (flags & hipEventDisableTiming) ? 1 : 0;
    if (used[k] < h->fev[k].size()) return h->fev[k][used[k]++];
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, flags) != hipSuccess) return nullptr;
    h->fev[k].push_back(e);
    ++used[k];
    return e;
  };
  // (the events stay in the handle's pool: every one this factorization
  // records is complete once the caller's stream has been synchronized)
#define STEP(...)                                                                 \
  do {                                                                            \
    hipError_t e_ = (__VA_ARGS__);                                                \
    if (e_ != hipSuccess) {                                                       \
      return fail_h(h, INVASKIT_E_HIP,                                            \
                    std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));    \
    }                                                                             \
  } while (0)
  // open(phase, stream) starts a bracket on a stream; close(stream) ends the
  // latest open bracket of that stream
  auto open = [&](int phase, hipStream_t st) -> hipError_t {
    hipEvent_t e = new_event(hipEventDefault);
    if (!e) return hipErrorOutOfMemory;
    brackets.push_back({e, nullptr, phase});
    open_on[st == s ? 0 : 1] = (int)brackets.size() - 1;
    return hipEventRecord(e, st);
  };
  auto close = [&](hipStream_t st) -> hipError_t {
    hipEvent_t e = new_event(hipEventDefault);
    if (!e) return hipErrorOutOfMemory;
    brackets[open_on[st == s ? 0 : 1]].b = e;
    return hipEventRecord(e, st);
  };
  // an event recorded on `st` now
  auto mark = [&](hipStream_t st, hipEvent_t* out) -> hipError_t {
    *out = new_event(hipEventDisableTiming);
    if (!*out) return hipErrorOutOfMemory;
    return hipEventRecord(*out, st);
  };
  // stream `to` waits for the work enqueued so far on `from`
  auto join = [&](hipStream_t from, hipStream_t to) -> hipError_t {
    hipEvent_t e = new_event(hipEventDisableTiming);
    if (!e) return hipErrorOutOfMemory;
    hipError_t r = hipEventRecord(e, from);
    return r == hipSuccess ? hipStreamWaitEvent(to, e, 0) : r;
  };
  const int L = h->L;
  // a plain plan settles its tiles first: the trials work in place on the
  // factor storage, and the factorization below starts from fresh blocks
  if (!fp.cached)
    if (int rc = tune_factor(h, fp)) return rc;
  hipEvent_t t_begin = new_event(hipEventDefault), t_end = new_event(hipEventDefault);
  if (!t_begin || !t_end) STEP(hipErrorOutOfMemory);
  STEP(hipEventRecord(t_begin, s));
  // the side stream starts after everything already on the caller's stream
  STEP(join(s, s2));
  const bool eval_now = !fp.cached || !kc->valid;
  hipEvent_t ev_panels = nullptr, ev_leaf = nullptr, ev_side = nullptr;
  // The skeleton blocks are first needed by the leaf solves.  A plain
  // factorization evaluates them on the side stream after the leaf blocks,
  // beside the large leaves' LU (latency-bound, it leaves the vector units
  // mostly idle), rather than beside the leaf blocks, which start the
  // critical path.  A sweep's cache is filled before anything else.
  const bool panels_late = eval_now && !fp.cached && L > 0;
  // the FP32 copy of P, first needed by the leaf projections, which wait
  // for the side stream
  auto convert_p = [&]() -> hipError_t {
    if (f64 || h->p_off[h->nn] <= 0) return hipSuccess;
    return launch_convert_f64_f32(h->P64, static_cast<float*>(const_cast<void*>(h->Pf)),
                                  h->p_off[h->nn], s2);
  };
  auto eval_panels = [&]() -> hipError_t {
    hipError_t e = open(3, s2);
    if (e == hipSuccess) e = run_eval(h, tb, fp.panels, 0.0, s2);
    if (e == hipSuccess) e = close(s2);
    if (e == hipSuccess) e = convert_p();
    return e == hipSuccess ? mark(s2, &ev_panels) : e;  // both are ready at ev_panels
  };
  if (eval_now) {
    // kernel blocks (into the factor storage, or once into a sweep's cache)
    if (L > 0 && !panels_late) STEP(eval_panels());
    if (L == 0) STEP(convert_p());
    STEP(open(0, s));
    STEP(run_eval(h, tb, fp.leaf_eval, fp.cached ? 0.0 : h->lam, s));
    STEP(close(s));
  }
  if (fp.cached) {
    if (eval_now) {
      STEP(join(s2, s));
      STEP(hipStreamSynchronize(s));
      kc->valid = true;
      ev_panels = nullptr;  // complete
    }
    // the tile choices need the evaluated cache (their trials copy from it)
    if (int rc = tune_factor(h, fp)) return rc;
    STEP(open(0, s));
    STEP(run_copy_shift(h, tb, fp.leaf_copy, s));
    STEP(close(s));
  }
  STEP(mark(s, &ev_leaf));  // every leaf block is in place
  auto lu_of = [&](const LuL& base) {
    LuL l = base;
    l.panel = h->tiles.leaf_lu_panel;
    l.waves = h->tiles.leaf_lu_waves;
    l.nopiv = h->leaf_nopiv;
    return l;
  };
  // small leaves on the second stream: LU, inverses and solves beside the
  // large leaves' LU, with the skeleton blocks between them unless they
  // were evaluated already
  const bool small = fp.leaf_lu[1].count > 0;
  if (small || panels_late) STEP(hipStreamWaitEvent(s2, ev_leaf, 0));
  if (small) {
    STEP(open(1, s2));
    STEP(run_lu(tb, lu_of(fp.leaf_lu[1]), s2));
    STEP(close(s2));
    STEP(open(2, s2));
    STEP(run_dinv(tb, fp.leaf_dinv[1], s2));
    STEP(close(s2));
  }
  if (panels_late) STEP(eval_panels());
  if (small && L > 0) {
    STEP(open(4, s2));
    STEP(run_trsm(tb, fp.leaf_trsm[1][h->tiles.leaf_trsm_cols_small == 32 ? 1 : 0], s2));
    STEP(close(s2));
    // the small leaves' projections, beside the large leaves' solves
    STEP(open(5, s2));
    STEP(run_gemm(tb, fp.leaf_proj[1], f64, s2));
    STEP(close(s2));
  }
  STEP(mark(s2, &ev_side));
  if (fp.leaf_lu[0].count > 0) {
    STEP(open(10, s));  // added into [1] below
    STEP(run_lu(tb, lu_of(fp.leaf_lu[0]), s));
    STEP(close(s));
    STEP(open(2, s));
    STEP(run_dinv(tb, fp.leaf_dinv[0], s));
    STEP(close(s));
  }
  if (L > 0) {
    if (ev_panels) STEP(hipStreamWaitEvent(s, ev_panels, 0));  // skeleton blocks done
    if (fp.leaf_lu[0].count > 0) {
      STEP(open(11, s));  // added into [4] below
      STEP(run_trsm(tb, fp.leaf_trsm[0][h->tiles.leaf_trsm_cols == 32 ? 1 : 0], s));
      STEP(close(s));
    }
  }
  if (L > 0) {
    STEP(open(12, s));  // added into [5] below
    STEP(run_gemm(tb, fp.leaf_proj[0], f64, s));
    STEP(close(s));
  }
  STEP(hipStreamWaitEvent(s, ev_side, 0));  // the small leaves are done
  if (L > 0) {
    // level wavefront
    for (int j = L - 1; j >= 0; --j) {
      int zf = kLuFormBlock, zc = kTrsmColsDefault;
      if (int rc = tune_level(h, tb, fp, j, s, &zf, &zc)) return rc;
      for (H* hg : hs) {
        if (zf == kLuFormOneWave) hg->tiles.zlu_one_wave_levels |= 1 << j;
        if (j >= 1 && zc == 32) hg->tiles.zsolve32_levels |= 1 << j;
      }
      LuL zl = fp.zlu[j];
      zl.form = zf;
      STEP(open(8, s));
      STEP(run_zform(tb, fp.zform[j], s));
      STEP(run_lu(tb, zl, s));
      STEP(run_dinv(tb, fp.zdinv[j], s));
      STEP(close(s));
      if (j >= 1) {
        STEP(open(6, s));
        STEP(run_trsm(tb, zc == 32 ? fp.zsolve32[j] : fp.zsolve[j], s));
        STEP(run_gemm(tb, fp.pgemm[j], f64, s));
        STEP(close(s));
      }
    }
  }
  STEP(hipEventRecord(t_end, s));
  for (size_t g = 0; g < hs.size(); ++g) {
    H* hg = hs[g];
    const size_t nz = info_at[g + 1] - info_at[g] - hg->nleaves;
    STEP(hipMemcpyAsync(info_host + info_at[g], hg->leafInfo.p, sizeof(int32_t) * hg->nleaves,
                        hipMemcpyDeviceToHost, s));
    if (nz > 0)
      STEP(hipMemcpyAsync(info_host + info_at[g] + hg->nleaves, hg->zinfo.p,
                          sizeof(int32_t) * nz, hipMemcpyDeviceToHost, s));
  }
  // each phase's time is read as soon as it has ended, while the GPU works
  // on the phases after it (the wavefront's levels), not all at the end
  double ms_ph[kPhases + 1] = {0};  // [12]: the large leaves' projections
  for (const Bracket& br : brackets) {
    if (!br.a || !br.b) continue;
    STEP(hipEventSynchronize(br.b));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, br.a, br.b) == hipSuccess) ms_ph[br.phase] += ms;
  }
  STEP(hipStreamSynchronize(s));
  {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t_begin, t_end) == hipSuccess) ms_ph[9] = ms;
  }
  // [1], [4] and [5] cover both size classes; [10], [11] and [12] the large
  // leaves alone
  ms_ph[1] += ms_ph[10];
  ms_ph[4] += ms_ph[11];
  ms_ph[5] += ms_ph[12];
#undef STEP
  // pivot status of every member
  int status = INVASKIT_OK;
  for (size_t g = 0; g < hs.size(); ++g) {
    H* hg = hs[g];
    for (int i = 0; i < kPhases; ++i) hg->phase_ms[i] = ms_ph[i];
    hg->phase_ms[7] = hg->plan_ms;
    hg->tiles = h->tiles;
    const int32_t* li = info_host + info_at[g];
    const int32_t* zi = li + hg->nleaves;
    const size_t nz = info_at[g + 1] - info_at[g] - hg->nleaves;
    int rc = INVASKIT_OK;
    for (int j = 0; j < hg->nleaves && !rc; ++j) {
      if (!li[j]) continue;
      if (h->leaf_nopiv) {
        // a pivot that is not positive: the block is not numerically
        // positive definite; the caller factors again with pivoting
        *repivot = true;
        break;
      }
      rc = fail_h(hg, INVASKIT_E_SINGULAR,
                  "zero pivot: leaf block of node " + std::to_string(hg->leaf_node(j)) +
                      " column " + std::to_string(li[j] - 1));
    }
    for (size_t a = 0; a < nz && !rc; ++a)
      if (zi[a])
        rc = fail_h(hg, INVASKIT_E_SINGULAR,
                    "zero pivot: reduced system of node " + std::to_string(a) + " column " +
                        std::to_string(zi[a] - 1));
    if (rc && status == INVASKIT_OK) status = rc;
  }
  return status;
}

// One factorization of the handles `hs` (one batched group): the leaf
// blocks without row exchanges when that is safe to try (leaf_pivoting
// AUTO and lambda > 0: lambda I + K_aa is then symmetric positive definite
// for the Gaussian kernel), again with partial pivoting if a pivot came out
// not positive.
int run_factor(const std::vector<H*>& hs, const FactorPlan& fp, KernelCache* kc) {
  bool nopiv = true;
  for (H* hg : hs) nopiv = nopiv && hg->leaf_pivoting == INVASKIT_LEAF_PIVOT_AUTO && hg->lam > 0.0;
  for (H* hg : hs) hg->leaf_nopiv = nopiv;
  bool repivot = false;
  int rc = run_factor_once(hs, fp, kc, &repivot);
  if (rc == INVASKIT_OK && repivot) {
    for (H* hg : hs) hg->leaf_nopiv = false;
    repivot = false;
    rc = run_factor_once(hs, fp, kc, &repivot);
  }
  for (H* hg : hs) hg->tiles.leaf_pivoting = hg->leaf_nopiv ? 0 : 1;
  return rc;
}

// ------------------------------------------------------------ solve plans
// Matvec tables (Skeletonize weights q = P [q_l; q_r] up the tree, then the
// fused Evaluate pass) for the plan's r columns, appended to `ar`.
void build_mv_tables(H* h, MatvecPlan& mp, Arena& ar) {
  const int L = h->L;
  const int r = mp.r;
  std::vector<int64_t> q_off(h->nn, 0);
  int64_t off = 0;
  for (int c = 1; c < h->nn; ++c) {
    q_off[c] = off;
    off += (int64_t)h->s[c] * r;
  }
  double* xm = static_cast<double*>(mp.xm.p);
  double* q = static_cast<double*>(mp.q.p);
  mp.skel.clear();
  for (int k = L; k >= 1; --k) {
    GemmBuilder gb;
    for (int c = (1 << k) - 1; c < (2 << k) - 1; ++c) {
      gb.begin(q + q_off[c], h->s[c], h->s[c], r, 1.0, 0.0);
      const double* Pc = h->P64 + h->p_off[c];
      if (k == L) {
        const int m = (int)(h->nb[c] - h->na[c]);
        gb.seg(Pc, m, true, xm + h->na[c], h->N, m);
      } else {
        const int l = 2 * c + 1, rr = 2 * c + 2;
        gb.seg(Pc, h->z[c], true, q + q_off[l], h->s[l], h->s[l]);
        gb.seg(Pc + h->s[l], h->z[c], true, q + q_off[rr], h->s[rr], h->s[rr]);
      }
    }
    mp.skel.push_back(gb.emit(ar));
  }
  // Evaluate: per leaf, its own block plus one skeleton segment per level
  std::vector<MvSeg> segs;
  std::vector<MvTile> tiles;
  for (int j = 0; j < h->nleaves; ++j) {
    const int lf = h->leaf_node(j);
    const int m = (int)(h->nb[lf] - h->na[lf]);
    const int seg0 = (int)segs.size();
    MvSeg g{};
    g.idx = nullptr;
    g.p0 = h->na[lf];
    g.w = xm + h->na[lf];
    g.ldw = h->N;
    g.count = m;
    segs.push_back(g);
    for (int k = 1; k <= L; ++k) {
      const int c = h->anc(lf, k);
      const int cs = h->sib(c);
      MvSeg t{};
      t.idx = h->skd + h->skel_off[cs];
      t.p0 = 0;
      t.w = q + q_off[cs];
      t.ldw = h->s[cs];
      t.count = h->s[cs];
      segs.push_back(t);
    }
    const int rows = h->d > kMvMaxDim ? kMvWideRows : kMvBlock;
    for (int t0 = 0; t0 < m; t0 += rows) {
      MvTile t{};
      t.row0 = h->na[lf] + t0;
      t.rows = std::min(rows, m - t0);
      t.seg0 = seg0;
      t.nseg = L + 1;
      tiles.push_back(t);
    }
  }
  mp.mv_segs = ar.add(segs);
  mp.mv_tiles = ar.add(tiles);
  mp.n_mv_tiles = (int)tiles.size();
}

int64_t skel_entries(const H* h) {  // sum of s_c over the non-root nodes
  int64_t t = 0;
  for (int c = 1; c < h->nn; ++c) t += h->s[c];
  return t;
}

// The plan of a solve (or, solve == false, of a matvec) with r right-hand
// sides whose scratch starts at `base`.  Scratch order: vectors, descriptor
// tables, then (solves) the GMRES bases, which a smaller scratch may leave
// out.
std::unique_ptr<SolvePlan> make_solve_plan(H* h, int r, bool solve, unsigned char* base) {
  auto sp = std::make_unique<SolvePlan>();
  sp->r = r;
  sp->solve = solve;
  sp->base = base;
  const int L = h->L;
  const size_t es = h->tsize();
  const int T64 = (h->prec == INVASKIT_PREC_FP64) ? 1 : 0;
  Carve cv;
  auto put = [&](Buf& b, size_t bytes) {
    const size_t o = cv.take(bytes);
    b.p = base + o;
    b.bytes = bytes;
  };
  const size_t nr = (size_t)h->N * r;
  std::vector<int64_t> sp_off(h->nn, 0), sy_off(h->nn, 0);
  int64_t off = 0;
  for (int c = 1; c < h->nn; ++c) {
    sp_off[c] = off;
    off += (int64_t)h->s[c] * r;
  }
  for (int c = 0; c < (1 << L) - 1; ++c) {
    sy_off[c] = off;
    off += (int64_t)h->z[c] * r;
  }
  if (solve) {
    put(sp->xbuf, nr * es);
    put(sp->sbuf, std::max<int64_t>(off, 1) * es);
    put(sp->x64, nr * 8);
    put(sp->r64, nr * 8);
    put(sp->sc, sizeof(double) * r);
    put(sp->gpart, sizeof(double) * dots_part_doubles(h->N, h->gm_restart + 1, r));
    put(sp->gsmall, sizeof(double) * (size_t)r * (4 * h->gm_restart + 3));
  }
  sp->mv.r = r;
  put(sp->mv.xm, nr * 8);
  put(sp->mv.q, std::max<int64_t>(skel_entries(h) * r, 1) * 8);
  Arena ar;
  if (solve) {
    void* xb = sp->xbuf.p;
    void* sb = sp->sbuf.p;
    const int32_t* lperm = static_cast<const int32_t*>(h->leafPerm.p);
    const int32_t* zpm = static_cast<const int32_t*>(h->zperm.p);
    TrsmBuilder lt;
    GemmBuilder lpj, fin;
    for (int j = 0; j < h->nleaves; ++j) {
      const int lf = h->leaf_node(j);
      const int m = (int)(h->nb[lf] - h->na[lf]);
      void* xr = offv(xb, h->na[lf], es);
      lt.add(offv(h->leafLU.p, h->lu_off[j], es), h->DL(j), lperm + h->na[lf], m, r, xr, h->N, m,
             xr, h->N, xr, h->N);
      if (L > 0) {
        lpj.begin(offv(sb, sp_off[lf], es), h->s[lf], h->s[lf], r, 1.0, 0.0);
        lpj.seg(offv(h->Pt(), h->p_off[lf], es), m, true, xr, h->N, m);
        fin.begin(xr, h->N, m, r, -1.0, 1.0);
        for (int jl = L; jl >= 1; --jl) {
          const int cj = h->anc(lf, jl);
          const int par = h->anc(lf, jl - 1);
          const int yoff = (cj & 1) ? 0 : h->s[cj];
          fin.seg(offv(h->slab.p, h->slab_off[j] + (int64_t)h->colk[j][jl] * m, es), m, false,
                  offv(sb, sy_off[par] + yoff, es), h->z[par], h->w[cj]);
        }
      }
    }
    sp->leaf_trsm = lt.emit(ar, T64, T64, 2);
    sp->leaf_proj = lpj.emit(ar);
    for (int jl = L - 1; jl >= 0; --jl) {
      TrsmBuilder zs;
      GemmBuilder pg;
      for (int bnode = (1 << jl) - 1; bnode < (2 << jl) - 1; ++bnode) {
        const int l = 2 * bnode + 1, rr = 2 * bnode + 2;
        void* y = offv(sb, sy_off[bnode], es);
        zs.add(h->Z(bnode), h->DZ(bnode), zpm + h->zperm_off[bnode], h->z[bnode], r,
               offv(sb, sp_off[rr], es), h->s[rr], h->s[rr], offv(sb, sp_off[l], es), h->s[l], y,
               h->z[bnode]);
        if (jl > 0) {
          pg.begin(offv(sb, sp_off[bnode], es), h->s[bnode], h->s[bnode], r, 1.0, 0.0);
          const void* Pb = offv(h->Pt(), h->p_off[bnode], es);
          pg.seg(Pb, h->z[bnode], true, offv(y, h->s[rr], es), h->z[bnode], h->s[l]);
          pg.seg(offv(Pb, h->s[l], es), h->z[bnode], true, y, h->z[bnode], h->s[rr]);
        }
      }
      sp->zsolve.push_back(zs.emit(ar, h->zis64[jl], T64, 2));
      sp->pgemm.push_back(pg.emit(ar));
    }
    // Top-down pass, levels i = 2 .. L: e_c = y^_c - sum_{j<i} Y^(i,j) e_{anc_j(c)},
    // in place of y^_c (the segment of the parent's solve y paired with the
    // sibling's skeleton).  Y^(i,j): rows of c in the parent's factor sweep
    // solution, columns of factor level j.  Level 1 needs no correction.
    const void* YS = h->ysw.p;
    auto yseg = [&](int c) {  // offset of c's segment inside its parent's y
      return (c & 1) ? 0 : h->s[c];
    };
    for (int i = 2; i <= L; ++i) {
      GemmBuilder td;
      for (int c = (1 << i) - 1; c < (2 << i) - 1; ++c) {
        const int par = (c - 1) / 2;
        const int wc = h->w[c];
        td.begin(offv(sb, sy_off[par] + yseg(c), es), h->z[par], wc, r, -1.0, 1.0);
        for (int j = 1; j < i; ++j) {
          const int cj = h->anc(c, j);
          const int pj = h->anc(c, j - 1);
          td.seg(offv(YS, h->ysw_off[par] + (int64_t)h->colp[par][j] * h->z[par] + yseg(c), es),
                 h->z[par], false, offv(sb, sy_off[pj] + yseg(cj), es), h->z[pj], h->w[cj]);
        }
      }
      sp->topdown.push_back(td.emit(ar));
    }
    sp->final_ = fin.emit(ar);
  }
  build_mv_tables(h, sp->mv, ar);
  put(sp->tables, ar.bytes());
  sp->blob = std::move(ar.host);
  sp->blob.resize(sp->tables.bytes, 0);
  sp->min_bytes = cv.total();
  if (solve) {
    sp->gm_m = h->gm_restart;
    put(sp->gmV, nr * 8 * (sp->gm_m + 1));
    put(sp->gmZ, nr * 8 * sp->gm_m);
  }
  sp->full_bytes = cv.total();
  return sp;
}

// The handle's plan for (r, solve) at scratch `base`, most recently used
// first; at most four are kept.
SolvePlan* get_solve_plan(H* h, int r, bool solve, unsigned char* base) {
  for (auto it = h->plans.begin(); it != h->plans.end(); ++it)
    if ((*it)->r == r && (*it)->solve == solve && (*it)->base == base) {
      if (it != h->plans.begin()) h->plans.splice(h->plans.begin(), h->plans, it);
      return h->plans.front().get();
    }
  h->plans.push_front(make_solve_plan(h, r, solve, base));
  while (h->plans.size() > 4) {
    if (h->up_plan == h->plans.back().get()) h->up_plan = nullptr;
    h->plans.pop_back();
  }
  return h->plans.front().get();
}

// Puts the plan's tables into the scratch unless they are already there
// (the previous call of this handle used the same plan and scratch).  For a
// solve, sets the GMRES bases the scratch has room for.
int bind_scratch(H* h, SolvePlan* sp, size_t scratch_bytes, bool force_upload) {
  if (sp->solve) {
    const size_t nr8 = (size_t)h->N * sp->r * 8;
    const size_t v0 = static_cast<unsigned char*>(sp->gmV.p) - static_cast<unsigned char*>(sp->base);
    sp->gm_m = 0;
    for (int m = h->gm_restart; m >= 2; --m) {
      const size_t need = v0 + align_up(nr8 * (m + 1), kAlign) + nr8 * m;
      if (need <= scratch_bytes) {
        sp->gm_m = m;
        break;
      }
    }
    if (sp->gm_m > 0)
      sp->gmZ.p = static_cast<unsigned char*>(sp->gmV.p) + align_up(nr8 * (sp->gm_m + 1), kAlign);
  }
  if (force_upload || h->up_plan != sp || h->up_base != sp->base) {
    HIP_TRY(h, hipMemcpyAsync(sp->tables.p, sp->blob.data(), sp->blob.size(),
                              hipMemcpyHostToDevice, h->stream));
    h->up_plan = force_upload ? nullptr : sp;
    h->up_base = sp->base;
  }
  return INVASKIT_OK;
}

// the direct solve on sp->xbuf, in place, in the factor precision
int run_solve_plan(H* h, SolvePlan* sp) {
  hipStream_t s = h->stream;
  const bool f64 = h->prec == INVASKIT_PREC_FP64;
  const Buf& tb = sp->tables;
  HIP_TRY(h, run_trsm(tb, sp->leaf_trsm, s));
  if (h->L == 0) return INVASKIT_OK;
  HIP_TRY(h, run_gemm(tb, sp->leaf_proj, f64, s));
  for (size_t q = 0; q < sp->zsolve.size(); ++q) {
    HIP_TRY(h, run_trsm(tb, sp->zsolve[q], s));
    HIP_TRY(h, run_gemm(tb, sp->pgemm[q], f64, s));
  }
  for (const GemmL& g : sp->topdown) HIP_TRY(h, run_gemm(tb, g, f64, s));
  HIP_TRY(h, run_gemm(tb, sp->final_, f64, s));
  return INVASKIT_OK;
}

// y = (lam I + K~) x  (or b - that when b != nullptr); x is copied first.
// With `overlap` (and d <= kMvMaxDim), the leaves' own blocks are summed on
// the side stream while the caller's stream forms the skeleton weights
// (Skeletonize), which only the other segments need; their raw sums wait
// in y and the second half continues from them in the same order, so the
// result is that of one whole pass bit for bit.
int run_matvec(H* h, const Buf& tb, const MatvecPlan& mp, const double* x, int64_t ldx, double* y,
               int64_t ldy, const double* b, int64_t ldb, bool overlap) {
  hipStream_t s = h->stream;
  const int r = mp.r;
  double* xm = static_cast<double*>(mp.xm.p);
  HIP_TRY(h, launch_copy_cols<double, double>(x, ldx, xm, h->N, h->N, r, nullptr, false, s));
  const MvTile* t = at<MvTile>(tb, mp.mv_tiles);
  const MvSeg* g = at<MvSeg>(tb, mp.mv_segs);
  auto eval = [&](int mode, hipStream_t st) -> hipError_t {
    if (h->pdt == INVASKIT_F64)
      return launch_mv_eval<double>(static_cast<const double*>(h->X), h->d, h->h, h->lam, t,
                                    mp.n_mv_tiles, g, xm, h->N, y, ldy, b, ldb, r, mode, st);
    return launch_mv_eval<float>(static_cast<const float*>(h->X), h->d, h->h, h->lam, t,
                                 mp.n_mv_tiles, g, xm, h->N, y, ldy, b, ldb, r, mode, st);
  };
  const bool split = overlap && h->side && h->L > 0 && h->d <= kMvMaxDim;
  if (split && !h->mv_ev[0]) {
    for (auto& e : h->mv_ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (split) {
    HIP_TRY(h, hipEventRecord(h->mv_ev[0], s));
    HIP_TRY(h, hipStreamWaitEvent(h->side, h->mv_ev[0], 0));
    HIP_TRY(h, eval(kMvNear, h->side));
    HIP_TRY(h, hipEventRecord(h->mv_ev[1], h->side));
  }
  for (const GemmL& gl : mp.skel) HIP_TRY(h, run_gemm(tb, gl, true, s));
  if (split) {
    HIP_TRY(h, hipStreamWaitEvent(s, h->mv_ev[1], 0));
    HIP_TRY(h, eval(kMvFar, s));
  } else {
    HIP_TRY(h, eval(kMvWhole, s));
  }
  return INVASKIT_OK;
}

// ------------------------------------------------------------ refinement
// Squared 2-norms of the r columns of an N x r FP64 block v (deterministic
// two-pass sums) into sp->gsmall[0, r) on the device and, for slot 0 or 1,
// copied on into the handle's pinned buffer at [slot * r, slot * r + r)
// (read after the stream is synchronized; slot -1: no copy).  The pinned
// buffer is reserved for two slots first.
int norms_back(H* h, SolvePlan* sp, int r, int slot);
int col_norms2_launch(H* h, SolvePlan* sp, const double* v, int64_t ld, int r, int slot) {
  double* part = static_cast<double*>(sp->gpart.p);
  double* out = static_cast<double*>(sp->gsmall.p);
  HIP_TRY(h, launch_dots(v, 0, ld, 1, v, ld, h->N, r, part, out, h->stream));
  return slot < 0 ? INVASKIT_OK : norms_back(h, sp, r, slot);
}

// the copy of sp->gsmall[0, r) into slot `slot` of the pinned buffer
int norms_back(H* h, SolvePlan* sp, int r, int slot) {
  const double* out = static_cast<const double*>(sp->gsmall.p);
  void* pin = nullptr;
  if (int rc = host_pinned(h, sizeof(double) * 2 * r, &pin)) return rc;
  HIP_TRY(h, hipMemcpyAsync(static_cast<double*>(pin) + (size_t)slot * r, out, sizeof(double) * r,
                            hipMemcpyDeviceToHost, h->stream));
  return INVASKIT_OK;
}

// the norms of slot `slot` once the stream has reached them
void pinned_norms(H* h, int r, int slot, std::vector<double>& host) {
  const double* p = static_cast<const double*>(h->pin) + (size_t)slot * r;
  host.assign(p, p + r);
}

// col_norms2_launch into slot 1, then a wait for the stream
int col_norms2(H* h, SolvePlan* sp, const double* v, int64_t ld, int r, std::vector<double>& host) {
  if (int rc = col_norms2_launch(h, sp, v, ld, r, 1)) return rc;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  pinned_norms(h, r, 1, host);
  return INVASKIT_OK;
}

// max over columns of |r_c| / |b_c| from squared norms (NaN propagates)
double worst_rel(const std::vector<double>& rn, const std::vector<double>& bn) {
  double worst = 0.0;
  for (size_t c = 0; c < rn.size(); ++c) {
    const double v = bn[c] > 0 ? std::sqrt(rn[c] / bn[c]) : std::sqrt(rn[c]);
    if (!(v <= worst)) worst = v;
  }
  return worst;
}

// One refinement step x64 += M^-1 res, with M^-1 the factors' direct
// solve (FP32 in mixed mode) and res the residual (r64; b itself for the
// first step, which sets x64 = M^-1 b instead of adding to it).  Each
// residual column is divided by its norm before the solve (so FP32 holds it
// at full relative precision) and the correction multiplied back.  The
// squared norms are those the last col_norms2_launch left in sp->gsmall
// (the residual's).
int ir_step(H* h, SolvePlan* sp, const double* res, int64_t ldres, bool first) {
  hipStream_t s = h->stream;
  const int r = sp->r;
  const int64_t N = h->N;
  double* x64 = static_cast<double*>(sp->x64.p);
  double* sc = static_cast<double*>(sp->sc.p);
  HIP_TRY(h, launch_sqrt_cols(static_cast<const double*>(sp->gsmall.p), sc, r, s));
  if (h->prec == INVASKIT_PREC_FP64) {
    double* xb = static_cast<double*>(sp->xbuf.p);
    HIP_TRY(h, launch_copy_cols<double, double>(res, ldres, xb, N, N, r, sc, true, s));
    if (int rc = run_solve_plan(h, sp)) return rc;
    if (first)
      HIP_TRY(h, launch_copy_cols<double, double>(xb, N, x64, N, N, r, sc, false, s));
    else
      HIP_TRY(h, launch_axpy_cols<double>(x64, N, xb, N, N, r, sc, s));
  } else {
    float* xb = static_cast<float*>(sp->xbuf.p);
    HIP_TRY(h, launch_copy_cols<double, float>(res, ldres, xb, N, N, r, sc, true, s));
    if (int rc = run_solve_plan(h, sp)) return rc;
    if (first)
      HIP_TRY(h, launch_copy_cols<float, double>(xb, N, x64, N, N, r, sc, false, s));
    else
      HIP_TRY(h, launch_axpy_cols<float>(x64, N, xb, N, N, r, sc, s));
  }
  return INVASKIT_OK;
}

// out = M^-1 in for unit-norm FP64 columns (a GMRES basis vector)
int apply_precond(H* h, SolvePlan* sp, const double* in, double* out) {
  hipStream_t s = h->stream;
  const int r = sp->r;
  const int64_t N = h->N;
  if (h->prec == INVASKIT_PREC_FP64) {
    double* xb = static_cast<double*>(sp->xbuf.p);
    HIP_TRY(h, launch_copy_cols<double, double>(in, N, xb, N, N, r, nullptr, false, s));
    if (int rc = run_solve_plan(h, sp)) return rc;
    HIP_TRY(h, launch_copy_cols<double, double>(xb, N, out, N, N, r, nullptr, false, s));
  } else {
    float* xb = static_cast<float*>(sp->xbuf.p);
    HIP_TRY(h, launch_copy_cols<double, float>(in, N, xb, N, N, r, nullptr, false, s));
    if (int rc = run_solve_plan(h, sp)) return rc;
    HIP_TRY(h, launch_copy_cols<float, double>(xb, N, out, N, N, r, nullptr, false, s));
  }
  return INVASKIT_OK;
}

// One cycle of restarted flexible GMRES (Saad's FGMRES) on A d = r64,
// right-preconditioned by M^-1, from d = 0, for every column at once (each
// column has its own Krylov space; they advance in lockstep).  Arnoldi with
// classical Gram-Schmidt applied twice.  Adds d to x64.  A column stops
// expanding its space when its least-squares residual estimate drops below
// est_tol[c] or the space becomes invariant.  Returns the steps taken in
// *steps (at most max_steps).
int gmres_cycle(H* h, SolvePlan* sp, const std::vector<double>& rn,
                const std::vector<double>& est_tol, int max_steps, int* steps) {
  hipStream_t s = h->stream;
  const int r = sp->r;
  const int m = std::min(sp->gm_m, max_steps);
  const int64_t N = h->N;
  const int64_t blk = N * r;  // one basis block: N x r, leading dimension N
  double* V = static_cast<double*>(sp->gmV.p);
  double* Zb = static_cast<double*>(sp->gmZ.p);
  double* x64 = static_cast<double*>(sp->x64.p);
  double* r64 = static_cast<double*>(sp->r64.p);
  double* part = static_cast<double*>(sp->gpart.p);
  double* small = static_cast<double*>(sp->gsmall.p);  // [h1 | h2 | nrm2 | coef]
  const int M1 = sp->gm_m + 1;
  double* h1d = small;
  double* h2d = small + (size_t)M1 * r;
  double* nrd = small + 2 * (size_t)M1 * r;
  double* cfd = small + 3 * (size_t)M1 * r;
  std::vector<double> H((size_t)r * M1 * m, 0.0), cs((size_t)r * m), sn((size_t)r * m);
  std::vector<double> g((size_t)r * M1, 0.0);
  std::vector<int> k(r, 0);
  std::vector<char> active(r, 0);
  std::vector<double> scale(r), hbuf(3 * (size_t)M1 * r);
  auto Hc = [&](int c, int i, int j) -> double& { return H[((size_t)c * M1 + i) * m + j]; };
  for (int c = 0; c < r; ++c) {
    const double beta = std::sqrt(rn[c]);
    g[(size_t)c * M1] = beta;
    active[c] = beta > est_tol[c];
    scale[c] = beta > 0 ? 1.0 / beta : 0.0;
  }
  HIP_TRY(h, hipMemcpyAsync(nrd, scale.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
  HIP_TRY(h, launch_copy_cols<double, double>(r64, N, V, N, N, r, nrd, false, s));
  HIP_TRY(h, hipStreamSynchronize(s));  // scale[] is rewritten below
  int j = 0;
  for (; j < m; ++j) {
    bool any = false;
    for (int c = 0; c < r; ++c) any = any || active[c];
    if (!any) break;
    double* vj = V + (size_t)j * blk;
    double* vn = V + (size_t)(j + 1) * blk;
    double* zj = Zb + (size_t)j * blk;
    if (int rc = apply_precond(h, sp, vj, zj)) return rc;
    if (int rc = run_matvec(h, sp->tables, sp->mv, zj, N, vn, N, nullptr, 0, true)) return rc;
    // classical Gram-Schmidt, twice
    HIP_TRY(h, launch_dots(V, blk, N, j + 1, vn, N, N, r, part, h1d, s));
    HIP_TRY(h, launch_lincomb(vn, N, V, blk, N, j + 1, h1d, r, -1.0, N, s));
    HIP_TRY(h, launch_dots(V, blk, N, j + 1, vn, N, N, r, part, h2d, s));
    HIP_TRY(h, launch_lincomb(vn, N, V, blk, N, j + 1, h2d, r, -1.0, N, s));
    HIP_TRY(h, launch_dots(vn, 0, N, 1, vn, N, N, r, part, nrd, s));
    HIP_TRY(h, hipMemcpyAsync(hbuf.data(), small, sizeof(double) * 3 * M1 * r,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    for (int c = 0; c < r; ++c) {
      scale[c] = 0.0;
      if (!active[c]) continue;
      double hn2 = 0.0;
      for (int i = 0; i <= j; ++i) {
        const double v = hbuf[(size_t)i * r + c] + hbuf[(size_t)M1 * r + (size_t)i * r + c];
        Hc(c, i, j) = v;
        hn2 += v * v;
      }
      const double hnext = std::sqrt(hbuf[2 * (size_t)M1 * r + c]);
      // rotations of the earlier columns, then a new one for row j + 1
      for (int i = 0; i < j; ++i) {
        const double a = Hc(c, i, j), b2 = Hc(c, i + 1, j);
        Hc(c, i, j) = cs[(size_t)c * m + i] * a + sn[(size_t)c * m + i] * b2;
        Hc(c, i + 1, j) = -sn[(size_t)c * m + i] * a + cs[(size_t)c * m + i] * b2;
      }
      const double a = Hc(c, j, j);
      const double dd = std::hypot(a, hnext);
      const double cj = dd > 0 ? a / dd : 1.0, sj = dd > 0 ? hnext / dd : 0.0;
      cs[(size_t)c * m + j] = cj;
      sn[(size_t)c * m + j] = sj;
      Hc(c, j, j) = dd;
      const double gj = g[(size_t)c * M1 + j];
      g[(size_t)c * M1 + j] = cj * gj;
      g[(size_t)c * M1 + j + 1] = -sj * gj;
      k[c] = j + 1;
      const bool invariant = !(hnext > 1e-14 * std::sqrt(hn2 + hnext * hnext));
      if (dd == 0.0 || !std::isfinite(dd)) {
        k[c] = j;  // no usable direction at this step
        active[c] = 0;
      } else if (invariant || std::fabs(g[(size_t)c * M1 + j + 1]) <= est_tol[c]) {
        active[c] = 0;
      } else {
        scale[c] = 1.0 / hnext;
      }
    }
    HIP_TRY(h, hipMemcpyAsync(nrd, scale.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
    HIP_TRY(h, launch_scale_cols(vn, N, N, r, nrd, s));
    HIP_TRY(h, hipStreamSynchronize(s));  // scale[] is rewritten next step
  }
  *steps = j;
  if (j == 0) return INVASKIT_OK;
  // y_c = R_c^-1 g_c (k_c x k_c upper triangle); zero beyond k_c
  std::vector<double> y((size_t)j * r, 0.0);
  for (int c = 0; c < r; ++c) {
    for (int i = k[c] - 1; i >= 0; --i) {
      double v = g[(size_t)c * M1 + i];
      for (int q = i + 1; q < k[c]; ++q) v -= Hc(c, i, q) * y[(size_t)q * r + c];
      y[(size_t)i * r + c] = v / Hc(c, i, i);
    }
  }
  HIP_TRY(h, hipMemcpyAsync(cfd, y.data(), sizeof(double) * y.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(h, launch_lincomb(x64, N, Zb, blk, N, j, cfd, r, 1.0, N, s));
  HIP_TRY(h, hipStreamSynchronize(s));  // y[] goes out of scope
  return INVASKIT_OK;
}

// The solve on a plan already bound to its scratch (bind_scratch).
int do_solve(H* h, SolvePlan* sp, const double* b, int64_t ldb, double* x, int64_t ldx,
             invaskit_solve_info* info) {
  const int r = sp->r;
  const int64_t N = h->N;
  hipStream_t s = h->stream;
  int rc;
  const int mode = h->refine;
  double* x64 = static_cast<double*>(sp->x64.p);
  double* r64 = static_cast<double*>(sp->r64.p);
  invaskit_solve_info loc{};
  loc.method = mode == INVASKIT_REFINE_NONE ? INVASKIT_REFINE_NONE : INVASKIT_REFINE_IR;
  std::vector<double> bn, rn;
  // The norms of b: the refinement reads them on the host only after its
  // first residual, which waits for the stream anyway, so they are copied
  // back without a wait of their own (slot 0), enqueued behind the first
  // step; a direct solve that reports nothing never reads them.  GMRES
  // from the start reads them at once.  The first step reads b itself and
  // sets x64 (GMRES sets up its own start).
  const bool bn_now = mode == INVASKIT_REFINE_GMRES;
  const bool bn_back = !bn_now && !(mode == INVASKIT_REFINE_NONE && !info);
  bool have_bn = bn_now;
  if (bn_now) {
    if ((rc = col_norms2(h, sp, b, ldb, r, bn))) return rc;
  } else {
    void* pin = nullptr;  // reserved before anything is in flight
    if (bn_back && (rc = host_pinned(h, sizeof(double) * 2 * r, &pin))) return rc;
    if ((rc = col_norms2_launch(h, sp, b, ldb, r, -1))) return rc;
  }
  rn = bn;
  // x = 0 is the first candidate (relative residual 1); the caller's x
  // always holds the best iterate so far
  double best = 1.0, prev = 1.0, hist[3] = {INFINITY, INFINITY, INFINITY};
  bool x_is_best_zero = true, last_is_best = true, conv = false, to_gmres = false;
  auto residual = [&]() -> int {  // r64 = b - A x64 and its norms
    int e = run_matvec(h, sp->tables, sp->mv, x64, N, r64, N, b, ldb, true);
    if (e) return e;
    if ((e = col_norms2(h, sp, r64, N, r, rn))) return e;
    if (!have_bn) {  // the stream has passed the copy of b's norms
      pinned_norms(h, r, 0, bn);
      have_bn = true;
    }
    return INVASKIT_OK;
  };
  auto keep_if_best = [&](double worst) -> int {
    last_is_best = worst < best;
    if (last_is_best) {
      best = worst;
      x_is_best_zero = false;
      HIP_TRY(h, launch_copy_cols<double, double>(x64, N, x, ldx, N, r, nullptr, false, s));
    }
    return INVASKIT_OK;
  };
  int it = 0;
  if (mode != INVASKIT_REFINE_GMRES) {
    const int cap = mode == INVASKIT_REFINE_NONE ? 1 : h->maxit;
    for (it = 1; it <= cap; ++it) {
      if ((rc = it == 1 ? ir_step(h, sp, b, ldb, true) : ir_step(h, sp, r64, N, false))) return rc;
      if (it == 1 && bn_back && (rc = norms_back(h, sp, r, 0))) return rc;
      if (mode == INVASKIT_REFINE_NONE && !info) {
        HIP_TRY(h, launch_copy_cols<double, double>(x64, N, x, ldx, N, r, nullptr, false, s));
        return INVASKIT_OK;
      }
      if ((rc = residual())) return rc;
      const double worst = worst_rel(rn, bn);
      if (it == 1) loc.unrefined_rel_residual = worst;
      if ((rc = keep_if_best(worst))) return rc;
      if (worst <= h->tol) {
        conv = true;
        break;
      }
      if (mode == INVASKIT_REFINE_NONE) break;
      if (mode == INVASKIT_REFINE_AUTO) {
        if (!(worst <= 0.5 * prev)) {  // not halved (or not finite): GMRES takes over
          to_gmres = true;
          break;
        }
      } else {
        if (!std::isfinite(worst)) break;
        // stall: no halving over the last three iterations
        if (it > 3 && worst > 0.5 * hist[0]) break;
        hist[0] = hist[1];
        hist[1] = hist[2];
        hist[2] = worst;
      }
      prev = worst;
    }
    loc.iterations = std::min(it, cap);
  }
  // without room for the GMRES bases (a scratch smaller than
  // invaskit_solve_workspace_bytes) AUTO ends with the refinement's best
  const bool no_room = sp->gm_m < 2;
  if (!conv && (mode == INVASKIT_REFINE_GMRES || to_gmres) && !no_room) {
    loc.method = INVASKIT_REFINE_GMRES;
    // restart from the best iterate
    if (x_is_best_zero) {
      HIP_TRY(h, launch_zero_cols(x64, N, N, r, s));
      HIP_TRY(h, launch_copy_cols<double, double>(b, ldb, r64, N, N, r, nullptr, false, s));
      rn = bn;
    } else if (!last_is_best) {
      HIP_TRY(h, launch_copy_cols<double, double>(x, ldx, x64, N, N, r, nullptr, false, s));
      if ((rc = residual())) return rc;
    }
    std::vector<double> est_tol(r);
    for (int c = 0; c < r; ++c) est_tol[c] = 0.1 * h->tol * std::sqrt(bn[c]);
    double cyc_prev = worst_rel(rn, bn);
    while (loc.gmres_iterations < h->gm_maxit) {
      int steps = 0;
      if ((rc = gmres_cycle(h, sp, rn, est_tol, h->gm_maxit - loc.gmres_iterations, &steps)))
        return rc;
      loc.gmres_iterations += steps;
      if ((rc = residual())) return rc;
      const double worst = worst_rel(rn, bn);
      if (mode == INVASKIT_REFINE_GMRES && loc.gmres_iterations == steps)
        loc.unrefined_rel_residual = worst;
      if ((rc = keep_if_best(worst))) return rc;
      if (worst <= h->tol) {
        conv = true;
        break;
      }
      // a cycle that gains less than 10% (or made no step) ends the solve
      if (steps == 0 || !(worst <= 0.9 * cyc_prev)) break;
      cyc_prev = worst;
    }
  }
  if (x_is_best_zero) HIP_TRY(h, launch_zero_cols(x, ldx, N, r, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  loc.converged = conv ? 1 : 0;
  loc.final_rel_residual = best;
  if (info) *info = loc;
  if (!conv)
    return fail_h(h, INVASKIT_E_NOT_CONVERGED,
                  "refinement stopped after " + std::to_string(loc.iterations) + " steps and " +
                      std::to_string(loc.gmres_iterations) +
                      " GMRES steps at relative residual " + std::to_string(best) +
                      (to_gmres && no_room ? " (no scratch for the GMRES bases)" : ""));
  return INVASKIT_OK;
}

// Address of this device's copy of `scratch`, looked up once per device
// with that device current.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // by device id

int static_scratch(H* h, unsigned char** out) {
  int dev = 0;
  HIP_TRY(h, hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail_h(h, INVASKIT_E_HIP,
                    std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return INVASKIT_OK;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

int invaskit_default_options(invaskit_options* opt) {
  if (!opt) return INVASKIT_E_ARG;
  opt->precision = INVASKIT_PREC_FP64;
  opt->fp64_top_levels = 4;
  opt->refine_tol = 1e-10;
  opt->max_refine_iters = 30;
  opt->tune = INVASKIT_TUNE_AUTO;
  opt->leaf_lu_panel = 0;
  opt->leaf_lu_waves = 0;
  opt->leaf_trsm_cols = 0;
  opt->refine = INVASKIT_REFINE_AUTO;
  opt->gmres_restart = 20;
  opt->max_gmres_iters = 300;
  opt->lambda_group = 0;
  opt->zlu_form = 0;
  opt->zsolve_cols = 0;
  opt->leaf_pivoting = INVASKIT_LEAF_PIVOT_AUTO;
  return INVASKIT_OK;
}

}  // extern "C"

namespace {
// A handle holding the validated problem's host description and options; no
// device access.
std::unique_ptr<H> new_handle(const invaskit_problem* pb, double lambda,
                              const invaskit_options* opt, void* hip_stream) {
  std::unique_ptr<H> h(new H());
  invaskit_options o;
  invaskit_default_options(&o);
  if (opt) o = *opt;
  h->prec = o.precision;
  h->top64 = o.fp64_top_levels;
  h->tol = o.refine_tol;
  h->maxit = o.max_refine_iters;
  h->tune = o.tune;
  h->fix_lu_panel = o.leaf_lu_panel;
  h->fix_lu_waves = o.leaf_lu_waves;
  h->fix_trsm_cols = o.leaf_trsm_cols;
  h->fix_zlu_form = o.zlu_form;
  h->fix_zsolve_cols = o.zsolve_cols;
  h->leaf_pivoting = o.leaf_pivoting;
  h->refine = o.refine;
  h->gm_restart = o.gmres_restart;
  h->gm_maxit = o.max_gmres_iters;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->N = pb->n;
  h->d = pb->d;
  h->L = pb->depth;
  h->pdt = pb->points_dtype;
  h->X = pb->points;
  h->P64 = pb->p_values;
  h->h = pb->h;
  h->lam = lambda;
  h->nleaves = 1 << h->L;
  h->nn = (1 << (h->L + 1)) - 1;
  h->leaf_off.assign(pb->leaf_offsets, pb->leaf_offsets + h->nleaves + 1);
  h->skel_off.assign(pb->skel_offsets, pb->skel_offsets + h->nn + 1);
  h->p_off.assign(pb->p_offsets, pb->p_offsets + h->nn + 1);
  if (h->skel_off[h->nn] > 0)
    h->skel_idx.assign(pb->skel_index, pb->skel_index + h->skel_off[h->nn]);
  layout_factor(h.get());
  return h;
}

// Sizes of one handle's region and of its own factor tables (placeholder
// base; shared: the sweep's cache, also at placeholder addresses).
void plan_region(H* h, const KernelCache* shared, size_t* region, size_t* tables) {
  carve_factor(h, kPlanBase, shared, 0);
  *tables = factor_table_bytes(h, shared);
  *region = carve_factor(h, kPlanBase, shared, *tables);
}

struct SweepSizes {
  size_t cache = 0, group_tables = 0, region = 0, single = 0, total = 0;
  int group = 1;
};
// Layout of a sweep's workspace: the shared cache, the tables of every
// lambda-batched group of two or more handles, then one region per handle.
SweepSizes sweep_sizes(H* h, int n_lambda, int lambda_group) {
  SweepSizes z;
  KernelCache kc;
  z.cache = carve_cache(h, kc, kPlanBase);
  plan_region(h, &kc, &z.region, &z.single);
  z.group = lambda_group > 0 ? std::min(lambda_group, n_lambda) : n_lambda;
  for (int i0 = 0; i0 < n_lambda; i0 += z.group) {
    const int g = std::min(z.group, n_lambda - i0);
    if (g >= 2) z.group_tables += align_up((size_t)g * z.single, kAlign);
  }
  z.total = z.cache + z.group_tables + (size_t)n_lambda * z.region;
  return z;
}

// Builds and uploads a handle's own factor plan (its tables in its region).
int ready_own_plan(H* h) {
  if (h->fp_ready) return INVASKIT_OK;
  Arena ar;
  build_factor_tables({h}, h->kcache.get(), ar, h->fp);
  if (ar.bytes() > h->fp.tables.bytes)
    return fail_h(h, INVASKIT_E_WORKSPACE, "internal: factor tables exceed their planned size");
  HIP_TRY(h, hipMemcpyAsync(h->fp.tables.p, ar.host.data(), ar.host.size(),
                            hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));  // ar goes out of scope
  h->fp_ready = true;
  return INVASKIT_OK;
}

// a cached plan carries lambda in its leaf copies: rewrite them
int set_plan_lambda(H* h) {
  const CopyShiftL& l = h->fp.leaf_copy;
  if (!h->fp.cached || l.count == 0) return INVASKIT_OK;
  std::vector<CopyShiftProb> c(l.count);
  CopyShiftProb* dev =
      reinterpret_cast<CopyShiftProb*>(static_cast<unsigned char*>(h->fp.tables.p) + l.probs);
  HIP_TRY(h, hipMemcpy(c.data(), dev, sizeof(CopyShiftProb) * c.size(), hipMemcpyDeviceToHost));
  for (auto& e : c) e.shift = h->lam;
  HIP_TRY(h, hipMemcpy(dev, c.data(), sizeof(CopyShiftProb) * c.size(), hipMemcpyHostToDevice));
  return INVASKIT_OK;
}
}  // namespace

extern "C" {

int invaskit_factor_workspace_bytes(const invaskit_problem* pb, const invaskit_options* opt,
                                    int32_t n_lambda, size_t* bytes) {
  if (!bytes) return fail_h(nullptr, INVASKIT_E_ARG, "bytes is NULL");
  if (n_lambda < 0) return fail_h(nullptr, INVASKIT_E_ARG, "n_lambda < 0");
  int rc = validate(nullptr, pb, 0.0, opt);
  if (rc) return rc;
  std::unique_ptr<H> h = new_handle(pb, 0.0, opt, nullptr);
  if (n_lambda == 0) {
    size_t region = 0, tables = 0;
    plan_region(h.get(), nullptr, &region, &tables);
    *bytes = region;
  } else {
    *bytes = sweep_sizes(h.get(), n_lambda, opt ? opt->lambda_group : 0).total;
  }
  return INVASKIT_OK;
}

int invaskit_factor(const invaskit_problem* pb, double lambda, const invaskit_options* opt,
                    void* workspace, size_t ws_bytes, void* hip_stream, invaskit_handle* out) {
  if (!out) return fail_h(nullptr, INVASKIT_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(nullptr, pb, lambda, opt);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<H> h = new_handle(pb, lambda, opt, hip_stream);
  // the tables come last in the region, so the other buffers' addresses are
  // final before the tables are built (once, with those addresses)
  unsigned char* base = static_cast<unsigned char*>(workspace);
  if (!base) return fail_h(nullptr, INVASKIT_E_ARG, "workspace is NULL");
  carve_factor(h.get(), base, nullptr, 0);
  Arena ar;
  build_factor_tables({h.get()}, nullptr, ar, h->fp);
  const size_t region = carve_factor(h.get(), base, nullptr, ar.bytes());
  if ((rc = check_workspace(nullptr, workspace, ws_bytes, region, "workspace"))) return rc;
  if ((rc = check_device(nullptr))) return rc;
  if (!h->skel_idx.empty())
    HIP_TRY(nullptr, hipMemcpyAsync(h->skel_own.p, h->skel_idx.data(),
                                    sizeof(int32_t) * h->skel_idx.size(), hipMemcpyHostToDevice,
                                    h->stream));
  HIP_TRY(nullptr, hipMemcpyAsync(h->fp.tables.p, ar.host.data(), ar.host.size(),
                                  hipMemcpyHostToDevice, h->stream));
  HIP_TRY(nullptr, hipStreamSynchronize(h->stream));  // ar goes out of scope
  h->fp_ready = true;
  h->plan_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  H* hp = h.get();
  rc = run_factor({hp}, hp->fp, nullptr);
  *out = h.release();
  return rc;
}

int invaskit_factor_sweep(const invaskit_problem* pb, const double* lambdas, int32_t n_lambda,
                          const invaskit_options* opt, void* workspace, size_t ws_bytes,
                          void* hip_stream, invaskit_handle* out) {
  if (!out || !lambdas || n_lambda < 1)
    return fail_h(nullptr, INVASKIT_E_ARG, "out, lambdas and n_lambda >= 1 are required");
  for (int32_t i = 0; i < n_lambda; ++i) out[i] = nullptr;
  for (int32_t i = 0; i < n_lambda; ++i) {
    int rc = validate(nullptr, pb, lambdas[i], opt);
    if (rc) return rc;
  }
  std::vector<std::unique_ptr<H>> hs;
  for (int32_t i = 0; i < n_lambda; ++i) hs.push_back(new_handle(pb, lambdas[i], opt, hip_stream));
  const SweepSizes z = sweep_sizes(hs[0].get(), n_lambda, opt ? opt->lambda_group : 0);
  int rc = check_workspace(nullptr, workspace, ws_bytes, z.total, "workspace");
  if (rc) return rc;
  if ((rc = check_device(nullptr))) return rc;
  unsigned char* base = static_cast<unsigned char*>(workspace);
  auto kc = std::make_shared<KernelCache>();
  carve_cache(hs[0].get(), *kc, base);
  unsigned char* gtab = base + z.cache;
  unsigned char* regions = gtab + z.group_tables;
  for (int32_t i = 0; i < n_lambda; ++i) {
    carve_factor(hs[i].get(), regions + (size_t)i * z.region, kc.get(), z.single);
    hs[i]->kcache = kc;
  }
  H* h0 = hs[0].get();
  if (!h0->skel_idx.empty())
    HIP_TRY(nullptr, hipMemcpyAsync(kc->skel.p, h0->skel_idx.data(),
                                    sizeof(int32_t) * h0->skel_idx.size(), hipMemcpyHostToDevice,
                                    h0->stream));
  int first = INVASKIT_OK;
  for (int32_t i0 = 0; i0 < n_lambda; i0 += z.group) {
    const int g = std::min(z.group, n_lambda - i0);
    const auto tb = std::chrono::steady_clock::now();
    std::vector<H*> members;
    for (int k = 0; k < g; ++k) members.push_back(hs[i0 + k].get());
    if (g == 1) {
      if ((rc = ready_own_plan(members[0]))) {
        first = rc;
        break;
      }
      members[0]->plan_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
      rc = run_factor(members, members[0]->fp, kc.get());
    } else {
      FactorPlan gp;
      gp.tables.p = gtab;
      gp.tables.bytes = align_up((size_t)g * z.single, kAlign);
      gtab += gp.tables.bytes;
      Arena ar;
      build_factor_tables(members, kc.get(), ar, gp);
      if (ar.bytes() > gp.tables.bytes) {
        first = fail_h(nullptr, INVASKIT_E_WORKSPACE,
                       "internal: sweep tables exceed their planned size");
        break;
      }
      hipError_t e = hipMemcpyAsync(gp.tables.p, ar.host.data(), ar.host.size(),
                                    hipMemcpyHostToDevice, h0->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h0->stream);
      if (e != hipSuccess) {
        first = fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
        break;
      }
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
      for (H* m : members) m->plan_ms = ms / g;
      rc = run_factor(members, gp, kc.get());
    }
    if (rc != INVASKIT_OK && first == INVASKIT_OK) first = rc;
    if (rc != INVASKIT_OK && rc != INVASKIT_E_SINGULAR) break;
  }
  if (first != INVASKIT_OK && first != INVASKIT_E_SINGULAR) {
    g_last_error = hs[0]->err.empty() ? g_last_error : hs[0]->err;
    return first;  // every handle is released
  }
  for (int32_t i = 0; i < n_lambda; ++i) out[i] = hs[i].release();
  if (first == INVASKIT_E_SINGULAR)
    for (int32_t i = 0; i < n_lambda; ++i)
      if (!out[i]->err.empty()) g_last_error = out[i]->err;
  return first;
}

int invaskit_refactor(invaskit_handle h, double lambda) {
  if (!h) return fail_h(nullptr, INVASKIT_E_ARG, "handle is NULL");
  if (!std::isfinite(lambda)) return fail_h(h, INVASKIT_E_ARG, "lambda must be finite");
  h->lam = lambda;
  int rc = ready_own_plan(h);
  if (!rc) rc = set_plan_lambda(h);
  if (rc) return rc;
  return run_factor({h}, h->fp, h->kcache.get());
}

int invaskit_solve_workspace_bytes(invaskit_handle h, int64_t nrhs, size_t* bytes,
                                   size_t* min_bytes) {
  if (!h || !bytes) return fail_h(h, INVASKIT_E_ARG, "handle and bytes are required");
  if (nrhs < 1 || nrhs > 4096) return fail_h(h, INVASKIT_E_ARG, "nrhs must be in [1, 4096]");
  const SolvePlan* sp = get_solve_plan(h, (int)nrhs, true, kPlanBase);
  *bytes = sp->full_bytes;
  if (min_bytes) *min_bytes = sp->min_bytes;
  return INVASKIT_OK;
}

int invaskit_matvec_workspace_bytes(invaskit_handle h, int64_t nrhs, size_t* bytes) {
  if (!h || !bytes) return fail_h(h, INVASKIT_E_ARG, "handle and bytes are required");
  if (nrhs < 1 || nrhs > 4096) return fail_h(h, INVASKIT_E_ARG, "nrhs must be in [1, 4096]");
  *bytes = get_solve_plan(h, (int)nrhs, false, kPlanBase)->full_bytes;
  return INVASKIT_OK;
}

int invaskit_solve(invaskit_handle h, const double* b, int64_t nrhs, int64_t ldb, double* x,
                   int64_t ldx, void* scratch, size_t scratch_bytes, invaskit_solve_info* info) {
  if (!h) return fail_h(nullptr, INVASKIT_E_ARG, "handle is NULL");
  if (!b || !x) return fail_h(h, INVASKIT_E_ARG, "b and x are required");
  if (nrhs < 1 || nrhs > 4096) return fail_h(h, INVASKIT_E_ARG, "nrhs must be in [1, 4096]");
  if (ldb < h->N || ldx < h->N) return fail_h(h, INVASKIT_E_ARG, "ldb and ldx must be >= n");
  const char* b0 = reinterpret_cast<const char*>(b);
  const char* b1 = reinterpret_cast<const char*>(b + (nrhs - 1) * ldb + h->N);
  const char* x0 = reinterpret_cast<const char*>(x);
  const char* x1 = reinterpret_cast<const char*>(x + (nrhs - 1) * ldx + h->N);
  if (b0 < x1 && x0 < b1) return fail_h(h, INVASKIT_E_ARG, "b and x overlap");
  if (!scratch) return fail_h(h, INVASKIT_E_ARG, "scratch is NULL");
  SolvePlan* sp = get_solve_plan(h, (int)nrhs, true, static_cast<unsigned char*>(scratch));
  int rc = check_workspace(h, scratch, scratch_bytes, sp->min_bytes, "scratch");
  if (rc) return rc;
  const char* s0 = static_cast<const char*>(scratch);
  if ((s0 < x1 && x0 < s0 + scratch_bytes) || (s0 < b1 && b0 < s0 + scratch_bytes))
    return fail_h(h, INVASKIT_E_ARG, "scratch overlaps b or x");
  if ((rc = bind_scratch(h, sp, scratch_bytes, false))) return rc;
  if (h->refine == INVASKIT_REFINE_GMRES && sp->gm_m < 2)
    return fail_h(h, INVASKIT_E_WORKSPACE,
                  "refine = GMRES needs the scratch size of invaskit_solve_workspace_bytes");
  return do_solve(h, sp, b, ldb, x, ldx, info);
}

int invaskit_matvec(invaskit_handle h, const double* x, int64_t nrhs, int64_t ldx, double* y,
                    int64_t ldy, void* scratch, size_t scratch_bytes) {
  if (!h) return fail_h(nullptr, INVASKIT_E_ARG, "handle is NULL");
  if (!x || !y) return fail_h(h, INVASKIT_E_ARG, "x and y are required");
  if (nrhs < 1 || nrhs > 4096) return fail_h(h, INVASKIT_E_ARG, "nrhs must be in [1, 4096]");
  if (ldx < h->N || ldy < h->N) return fail_h(h, INVASKIT_E_ARG, "ldx and ldy must be >= n");
  if (!scratch) return fail_h(h, INVASKIT_E_ARG, "scratch is NULL");
  SolvePlan* sp = get_solve_plan(h, (int)nrhs, false, static_cast<unsigned char*>(scratch));
  int rc = check_workspace(h, scratch, scratch_bytes, sp->min_bytes, "scratch");
  if (rc) return rc;
  if ((rc = bind_scratch(h, sp, scratch_bytes, false))) return rc;
  return run_matvec(h, sp->tables, sp->mv, x, ldx, y, ldy, nullptr, 0, true);
}

int invaskit_matvec_noalloc(invaskit_handle h, const double* x, int64_t nrhs, int64_t ldx,
                            double* y, int64_t ldy) {
  if (!h) return fail_h(nullptr, INVASKIT_E_ARG, "handle is NULL");
  if (!x || !y) return fail_h(h, INVASKIT_E_ARG, "x and y are required");
  if (nrhs < 1 || nrhs > 4096) return fail_h(h, INVASKIT_E_ARG, "nrhs must be in [1, 4096]");
  if (ldx < h->N || ldy < h->N) return fail_h(h, INVASKIT_E_ARG, "ldx and ldy must be >= n");
  unsigned char* base = nullptr;
  int rc = static_scratch(h, &base);
  if (rc) return rc;
  SolvePlan* sp = get_solve_plan(h, (int)nrhs, false, base);
  if (sp->min_bytes > (size_t)INVASKIT_STATIC_SCRATCH_BYTES)
    return fail_h(h, INVASKIT_E_WORKSPACE,
                  "this product needs " + std::to_string(sp->min_bytes) +
                      " bytes of scratch; the static scratch holds " +
                      std::to_string((size_t)INVASKIT_STATIC_SCRATCH_BYTES));
  // other handles may have used the array since: always copy the tables
  if ((rc = bind_scratch(h, sp, INVASKIT_STATIC_SCRATCH_BYTES, true))) return rc;
  // one stream, one pass: nothing beyond the caller's stream is involved
  return run_matvec(h, sp->tables, sp->mv, x, ldx, y, ldy, nullptr, 0, false);
}

int invaskit_device_bytes(invaskit_handle h, size_t* bytes) {
  if (!h || !bytes) return fail_h(h, INVASKIT_E_ARG, "handle and bytes are required");
  *bytes = h->region_bytes;
  return INVASKIT_OK;
}

int invaskit_phase_times(invaskit_handle h, double* ms, int32_t n) {
  if (!h || !ms) return fail_h(h, INVASKIT_E_ARG, "handle and ms are required");
  for (int i = 0; i < std::min(n, kPhases); ++i) ms[i] = h->phase_ms[i];
  return INVASKIT_OK;
}

int invaskit_tile_config_get(invaskit_handle h, invaskit_tile_config* out) {
  if (!h || !out) return fail_h(h, INVASKIT_E_ARG, "handle and out are required");
  *out = h->tiles;
  return INVASKIT_OK;
}

int invaskit_tuning_export(char* buf, size_t n, size_t* needed) {
  if (!needed || (n > 0 && !buf)) return fail_h(nullptr, INVASKIT_E_ARG, "needed is required");
  std::string text;
  {
    std::lock_guard<std::mutex> g(tune_table().mu);
    for (const auto& kv : tune_table().choice)
      text += kv.first + " " + std::to_string(kv.second) + "\n";
  }
  *needed = text.size() + 1;
  if (n > 0) {
    const size_t k = std::min(n - 1, text.size());
    std::memcpy(buf, text.data(), k);
    buf[k] = '\0';
  }
  return INVASKIT_OK;
}

int invaskit_tuning_import(const char* text) {
  if (!text) return fail_h(nullptr, INVASKIT_E_ARG, "text is NULL");
  std::vector<std::pair<std::string, int>> add;
  std::istringstream in(text);
  std::string line;
  while (std::getline(in, line)) {
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    std::istringstream ls(line);
    std::string key, rest;
    int v = 0;
    const bool parsed = (ls >> key >> v) && !(ls >> rest);
    const bool waves = key.rfind("getrfw.", 0) == 0;
    const bool tile = key.rfind("getrf.", 0) == 0 || key.rfind("getrs.", 0) == 0;
    const bool zform = key.rfind("zgetrf.", 0) == 0;
    if (!parsed || !(waves || tile || zform) || (waves && v != 4 && v != 8) ||
        (tile && v != 16 && v != 32) ||
        (zform && v != kLuFormOneWave && v != kLuFormBlock))
      return fail_h(nullptr, INVASKIT_E_ARG, "malformed tuning line: " + line);
    add.emplace_back(key, v);
  }
  std::lock_guard<std::mutex> g(tune_table().mu);
  for (const auto& kv : add) tune_table().choice[kv.first] = kv.second;
  return INVASKIT_OK;
}

int invaskit_tuning_clear(void) {
  std::lock_guard<std::mutex> g(tune_table().mu);
  tune_table().choice.clear();
  return INVASKIT_OK;
}

int invaskit_destroy(invaskit_handle h) {
  if (!h) return INVASKIT_OK;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return INVASKIT_OK;
}

const char* invaskit_status_string(int status) {
  switch (status) {
    case INVASKIT_OK: return "ok";
    case INVASKIT_E_ARG: return "invalid argument";
    case INVASKIT_E_WORKSPACE: return "workspace too small";
    case INVASKIT_E_HIP: return "HIP runtime error";
    case INVASKIT_E_SINGULAR: return "singular pivot";
    case INVASKIT_E_NOT_CONVERGED: return "refinement did not converge";
    case INVASKIT_E_DEVICE: return "no usable gfx950 device";
    default: return "unknown status";
  }
}

int invaskit_last_error(invaskit_handle h, char* buf, size_t n) {
  if (!buf || n == 0) return INVASKIT_E_ARG;
  const std::string& m = h ? h->err : g_last_error;
  const size_t k = std::min(n - 1, m.size());
  std::memcpy(buf, m.data(), k);
  buf[k] = 0;
  return INVASKIT_OK;
}

// ----------------------------------------------------- batched building blocks
}  // extern "C"

namespace {
// A building block's device memory: `need` bytes of the caller's workspace.
// With workspace == NULL the call only reports the size (*ws_needed).
int block_workspace(void* ws, size_t ws_bytes, size_t* ws_needed, size_t need, bool* query) {
  if (ws_needed) *ws_needed = need;
  *query = ws == nullptr;
  if (!ws)
    return ws_needed ? INVASKIT_OK
                     : fail_h(nullptr, INVASKIT_E_ARG, "workspace and ws_needed are both NULL");
  return check_workspace(nullptr, ws, ws_bytes, need, "workspace");
}

int upload_and_sync(const Arena& ar, void* dst, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst, ar.host.data(), ar.host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
  return INVASKIT_OK;
}
}  // namespace

extern "C" {

int invaskit_getrf_batched(int32_t dtype, void* a, const int64_t* a_offsets, const int32_t* n,
                           int32_t count, int32_t* perm, int32_t* info, void* workspace,
                           size_t ws_bytes, size_t* ws_needed, void* hip_stream) {
  if (count < 0 || (count > 0 && (!a || !a_offsets || !n || !perm || !info)))
    return fail_h(nullptr, INVASKIT_E_ARG, "invalid getrf_batched arguments");
  if (dtype != INVASKIT_F64 && dtype != INVASKIT_F32)
    return fail_h(nullptr, INVASKIT_E_ARG, "dtype must be INVASKIT_F64 or INVASKIT_F32");
  const size_t es = dtype == INVASKIT_F64 ? 8 : 4;
  Arena ar;
  std::vector<LuProb> probs(count);
  int nmax = 0;
  int64_t poff = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kMaxLeaf) return fail_h(nullptr, INVASKIT_E_ARG, "n out of range");
    probs[i].a = static_cast<unsigned char*>(a) + a_offsets[i] * es;
    probs[i].perm = perm + poff;
    probs[i].info = info + i;
    probs[i].n = n[i];
    poff += n[i];
    nmax = std::max(nmax, n[i]);
  }
  const size_t off = ar.add(probs);
  bool query = false;
  int rc = block_workspace(workspace, ws_bytes, ws_needed, ar.bytes(), &query);
  if (rc || query || count == 0) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = upload_and_sync(ar, workspace, s))) return rc;
  const LuProb* t = reinterpret_cast<const LuProb*>(static_cast<unsigned char*>(workspace) + off);
  hipError_t e = (dtype == INVASKIT_F64) ? launch_getrf<double>(t, count, nmax, 1, 0, 0, s)
                                         : launch_getrf<float>(t, count, nmax, 1, 0, 0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
  return INVASKIT_OK;
}

}  // extern "C"

namespace {
// Tables of a batched solve with caller-owned factors; the diagonal-block
// inverses go at the start of `base`, the tables after them.
int getrs_tables(int32_t dtype, const void* a, const int64_t* a_offsets, const int32_t* n,
                 const int32_t* perm, void* b, const int64_t* b_offsets, const int32_t* nrhs,
                 const int64_t* ldb, int32_t count, unsigned char* base, Arena& ar, size_t* tables,
                 TrsmL* l, DinvL* dl) {
  const size_t es = dtype == INVASKIT_F64 ? 8 : 4;
  constexpr int64_t kDB2 = 2 * kDiagBlock * kDiagBlock;
  int64_t dn = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kMaxLeaf || nrhs[i] < 0 || ldb[i] < n[i])
      return fail_h(nullptr, INVASKIT_E_ARG, "getrs_batched sizes out of range");
    dn += (n[i] + kDiagBlock - 1) / kDiagBlock * kDB2;
  }
  *tables = align_up(std::max<int64_t>(dn, 1) * es, kAlign);
  TrsmBuilder tb;
  std::vector<DiagInvProb> dis;
  int64_t poff = 0, doff = 0;
  for (int i = 0; i < count; ++i) {
    const unsigned char* ai = static_cast<const unsigned char*>(a) + a_offsets[i] * es;
    void* di = base + doff * es;
    for (int jb = 0; jb < n[i]; jb += kDiagBlock) {
      DiagInvProb d{};
      d.lu = ai;
      d.perm = perm + poff;
      d.out = static_cast<unsigned char*>(di) + (jb / kDiagBlock) * kDB2 * es;
      d.n = n[i];
      d.jb = jb;
      dis.push_back(d);
    }
    void* bi = static_cast<unsigned char*>(b) + b_offsets[i] * es;
    tb.add(ai, di, perm + poff, n[i], nrhs[i], bi, ldb[i], n[i], bi, ldb[i], bi, ldb[i]);
    poff += n[i];
    doff += (n[i] + kDiagBlock - 1) / kDiagBlock * kDB2;
  }
  const int f = dtype == INVASKIT_F64 ? 1 : 0;
  *l = tb.emit(ar, f, f, 3);  // caller-owned factors: checked loads
  dl->probs = ar.add(dis);
  dl->count = (int)dis.size();
  dl->t64 = f;
  return INVASKIT_OK;
}
}  // namespace

extern "C" {

int invaskit_getrs_batched(int32_t dtype, const void* a, const int64_t* a_offsets,
                           const int32_t* n, const int32_t* perm, void* b,
                           const int64_t* b_offsets, const int32_t* nrhs, const int64_t* ldb,
                           int32_t count, void* workspace, size_t ws_bytes, size_t* ws_needed,
                           void* hip_stream) {
  if (count < 0 || (count > 0 && (!a || !a_offsets || !n || !perm || !b || !b_offsets || !nrhs ||
                                  !ldb)))
    return fail_h(nullptr, INVASKIT_E_ARG, "invalid getrs_batched arguments");
  if (dtype != INVASKIT_F64 && dtype != INVASKIT_F32)
    return fail_h(nullptr, INVASKIT_E_ARG, "dtype must be INVASKIT_F64 or INVASKIT_F32");
  unsigned char* base = workspace ? static_cast<unsigned char*>(workspace) : kPlanBase;
  Arena ar;
  size_t dbytes = 0;
  TrsmL l;
  DinvL dl;
  int rc = getrs_tables(dtype, a, a_offsets, n, perm, b, b_offsets, nrhs, ldb, count, base, ar,
                        &dbytes, &l, &dl);
  if (rc) return rc;
  bool query = false;
  rc = block_workspace(workspace, ws_bytes, ws_needed, dbytes + ar.bytes(), &query);
  if (rc || query || count == 0) return rc;
  if (l.ntiles < 0)
    return fail_h(nullptr, INVASKIT_E_ARG, "getrs_batched: the largest system needs too much LDS");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Buf t{base + dbytes, ar.bytes()};
  if ((rc = upload_and_sync(ar, t.p, s))) return rc;
  hipError_t e = run_dinv(t, dl, s);
  if (e == hipSuccess) e = run_trsm(t, l, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
  return INVASKIT_OK;
}

int invaskit_kernel_blocks(int32_t points_dtype, const void* points, int32_t d, double hbw,
                           int32_t out_dtype, void* out, const int64_t* out_offsets,
                           const int64_t* row0, const int32_t* rows, const int32_t* cols,
                           const int64_t* cols_offsets, const int32_t* ncols, const int32_t* diag,
                           double shift, int32_t count, void* workspace, size_t ws_bytes,
                           size_t* ws_needed, void* hip_stream) {
  if (count < 0 || d < 1 || !(hbw > 0) ||
      (count > 0 && (!points || !out || !out_offsets || !row0 || !rows || !cols ||
                     !cols_offsets || !ncols || !diag)))
    return fail_h(nullptr, INVASKIT_E_ARG, "invalid kernel_blocks arguments");
  if ((points_dtype != INVASKIT_F64 && points_dtype != INVASKIT_F32) ||
      (out_dtype != INVASKIT_F64 && out_dtype != INVASKIT_F32))
    return fail_h(nullptr, INVASKIT_E_ARG, "dtypes must be INVASKIT_F64 or INVASKIT_F32");
  const size_t es = out_dtype == INVASKIT_F64 ? 8 : 4;
  std::vector<EvalBlock> blocks(count);
  std::vector<Tile3> tiles;
  for (int i = 0; i < count; ++i) {
    if (rows[i] < 0 || ncols[i] < 0) return fail_h(nullptr, INVASKIT_E_ARG, "negative block size");
    EvalBlock& b = blocks[i];
    b.out = static_cast<unsigned char*>(out) + out_offsets[i] * es;
    b.ld = rows[i];
    b.row0 = row0[i];
    b.cols = cols + cols_offsets[i];
    b.col0 = 0;
    b.rows = rows[i];
    b.ncols = ncols[i];
    b.diag = diag[i];
    for (int tn = 0; tn < (ncols[i] + kEvalTile - 1) / kEvalTile; ++tn)
      for (int tm = 0; tm < (rows[i] + kEvalTile - 1) / kEvalTile; ++tm) tiles.push_back({i, tm, tn});
  }
  Arena ar;
  const size_t ob = ar.add(blocks), ot = ar.add(tiles);
  bool query = false;
  int rc = block_workspace(workspace, ws_bytes, ws_needed, ar.bytes(), &query);
  if (rc || query || count == 0) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = upload_and_sync(ar, workspace, s))) return rc;
  Buf t{workspace, ar.bytes()};
  const int nt = (int)tiles.size();
  const EvalBlock* pb = at<EvalBlock>(t, ob);
  const Tile3* pt = at<Tile3>(t, ot);
  hipError_t e;
  if (points_dtype == INVASKIT_F64) {
    const double* X = static_cast<const double*>(points);
    e = out_dtype == INVASKIT_F64 ? launch_eval<double, double>(X, d, hbw, shift, pb, pt, nt, s)
                                  : launch_eval<double, float>(X, d, hbw, shift, pb, pt, nt, s);
  } else {
    const float* X = static_cast<const float*>(points);
    e = out_dtype == INVASKIT_F64 ? launch_eval<float, double>(X, d, hbw, shift, pb, pt, nt, s)
                                  : launch_eval<float, float>(X, d, hbw, shift, pb, pt, nt, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
  return INVASKIT_OK;
}

int invaskit_gemm_batched(int32_t dtype, const void* a, const void* b, void* c,
                          const int64_t* a_off, const int64_t* b_off, const int64_t* c_off,
                          const int32_t* m, const int32_t* n, const int32_t* k,
                          const int64_t* lda, const int32_t* a_rm, const int64_t* ldb,
                          const int64_t* ldc, double alpha, double beta, int32_t count,
                          void* workspace, size_t ws_bytes, size_t* ws_needed, void* hip_stream) {
  if (count < 0 || (count > 0 && (!a || !b || !c || !a_off || !b_off || !c_off || !m || !n ||
                                  !k || !lda || !a_rm || !ldb || !ldc)))
    return fail_h(nullptr, INVASKIT_E_ARG, "invalid gemm_batched arguments");
  if (dtype != INVASKIT_F64 && dtype != INVASKIT_F32)
    return fail_h(nullptr, INVASKIT_E_ARG, "dtype must be INVASKIT_F64 or INVASKIT_F32");
  const size_t es = dtype == INVASKIT_F64 ? 8 : 4;
  GemmBuilder gb;
  for (int i = 0; i < count; ++i) {
    if (m[i] < 0 || n[i] < 0 || k[i] < 0 || ldc[i] < m[i] || ldb[i] < k[i] ||
        lda[i] < (a_rm[i] ? k[i] : m[i]))
      return fail_h(nullptr, INVASKIT_E_ARG, "gemm_batched sizes out of range");
    gb.begin(static_cast<unsigned char*>(c) + c_off[i] * es, ldc[i], m[i], n[i], alpha, beta);
    gb.seg(static_cast<const unsigned char*>(a) + a_off[i] * es, lda[i], a_rm[i] != 0,
           static_cast<const unsigned char*>(b) + b_off[i] * es, ldb[i], k[i]);
  }
  Arena ar;
  GemmL l = gb.emit(ar);
  bool query = false;
  int rc = block_workspace(workspace, ws_bytes, ws_needed, ar.bytes(), &query);
  if (rc || query || count == 0) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = upload_and_sync(ar, workspace, s))) return rc;
  Buf t{workspace, ar.bytes()};
  hipError_t e = run_gemm(t, l, dtype == INVASKIT_F64, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_h(nullptr, INVASKIT_E_HIP, hipGetErrorString(e));
  return INVASKIT_OK;
}

}  // extern "C"

