// Host-only driver for the sanitizer build of the library's host code: plans
// the workspace of many synthetic problems (uneven leaves, ragged nested
// skeletons, every depth from 0 to 7, both precisions, sweeps and lambda
// groups), rejects malformed ones, and queries the building blocks'
// workspaces.  No device is touched; a factorization stops at its device
// check after validation and planning.  Exit status 0 when every call
// returned what the case expects.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "invaskit.h"

namespace {

struct Tree {
  int depth = 0;
  int64_t n = 0;
  std::vector<int64_t> leaf, so, po;
  std::vector<int32_t> si;
};

// A complete tree of the given depth with leaves of 1..max_leaf points and
// nested skeletons: a leaf keeps a random subset of its points, an internal
// node a random subset of its children's skeletons.
Tree make_tree(int depth, int max_leaf, int max_skel, std::mt19937& g) {
  Tree t;
  t.depth = depth;
  const int nleaves = 1 << depth, nn = (1 << (depth + 1)) - 1;
  t.leaf.assign(nleaves + 1, 0);
  for (int j = 0; j < nleaves; ++j)
    t.leaf[j + 1] = t.leaf[j] + 1 + (int64_t)(g() % (unsigned)max_leaf);
  t.n = t.leaf[nleaves];
  std::vector<std::vector<int32_t>> sk(nn);
  for (int c = nn - 1; c >= 1; --c) {
    std::vector<int32_t> cand;
    if (c >= nleaves - 1) {
      const int j = c - (nleaves - 1);
      for (int64_t i = t.leaf[j]; i < t.leaf[j + 1]; ++i) cand.push_back((int32_t)i);
    } else {
      cand = sk[2 * c + 1];
      cand.insert(cand.end(), sk[2 * c + 2].begin(), sk[2 * c + 2].end());
    }
    std::shuffle(cand.begin(), cand.end(), g);
    const int s = 1 + (int)(g() % (unsigned)std::min<size_t>(cand.size(), (size_t)max_skel));
    sk[c].assign(cand.begin(), cand.begin() + s);
  }
  t.so.assign(nn + 1, 0);
  t.po.assign(nn + 1, 0);
  for (int c = 0; c < nn; ++c) {
    t.so[c + 1] = t.so[c] + (int64_t)sk[c].size();
    t.si.insert(t.si.end(), sk[c].begin(), sk[c].end());
    int64_t cols = 0;
    if (c > 0) {
      if (c >= nleaves - 1) {
        const int j = c - (nleaves - 1);
        cols = t.leaf[j + 1] - t.leaf[j];
      } else {
        cols = (int64_t)sk[2 * c + 1].size() + (int64_t)sk[2 * c + 2].size();
      }
    }
    t.po[c + 1] = t.po[c] + (int64_t)sk[c].size() * cols;
  }
  return t;
}

invaskit_problem problem_of(const Tree& t) {
  invaskit_problem p{};
  p.n = t.n;
  p.d = 5;
  p.depth = t.depth;
  p.points_dtype = INVASKIT_F64;
  p.points = reinterpret_cast<const void*>(uintptr_t(1) << 20);  // never dereferenced
  p.leaf_offsets = t.leaf.data();
  p.skel_offsets = t.so.data();
  p.skel_index = t.si.data();
  p.p_offsets = t.po.data();
  p.p_values = reinterpret_cast<const double*>(uintptr_t(2) << 20);
  p.h = 1.0;
  return p;
}

int failures = 0;
void expect(bool ok, const char* what, int depth) {
  if (!ok) {
    ++failures;
    std::fprintf(stderr, "FAILED: %s (depth %d)\n", what, depth);
  }
}

}  // namespace

int main() {
  std::mt19937 g(20261203);
  for (int rep = 0; rep < 3; ++rep) {
    for (int depth = 0; depth <= 7; ++depth) {
      const Tree t = make_tree(depth, depth < 4 ? 300 : 80, depth < 4 ? 90 : 40, g);
      const invaskit_problem pb = problem_of(t);
      for (int prec : {INVASKIT_PREC_FP64, INVASKIT_PREC_MIXED}) {
        invaskit_options o;
        invaskit_default_options(&o);
        o.precision = prec;
        o.fp64_top_levels = (int)(g() % 5);
        size_t one = 0, sweep = 0, grouped = 0;
        expect(invaskit_factor_workspace_bytes(&pb, &o, 0, &one) == INVASKIT_OK && one > 0,
               "workspace of one factorization", depth);
        expect(invaskit_factor_workspace_bytes(&pb, &o, 3, &sweep) == INVASKIT_OK &&
                   sweep > one, "workspace of a sweep", depth);
        o.lambda_group = 1;
        expect(invaskit_factor_workspace_bytes(&pb, &o, 3, &grouped) == INVASKIT_OK &&
                   grouped <= sweep, "workspace of a sweep in groups of one", depth);
        o.lambda_group = 0;
        // too small: refused before any device access
        invaskit_handle h = nullptr;
        void* fake = reinterpret_cast<void*>(uintptr_t(1) << 30);
        expect(invaskit_factor(&pb, 1e-2, &o, fake, one - 1, nullptr, &h) ==
                   INVASKIT_E_WORKSPACE && h == nullptr, "short workspace", depth);
        // large enough: validation and planning pass, the device check fails
        // on a machine without a gfx950 GPU (no handle is returned)
        const int st = invaskit_factor(&pb, 1e-2, &o, fake, one, nullptr, &h);
        expect(st != INVASKIT_OK && st != INVASKIT_E_ARG && st != INVASKIT_E_WORKSPACE &&
                   h == nullptr, "device check after planning", depth);
      }
      {
        // a sweep of three lambdas: sizes, carving and the device check
        invaskit_options o;
        invaskit_default_options(&o);
        o.precision = INVASKIT_PREC_MIXED;
        o.lambda_group = 2;
        const double lam[3] = {1e-3, 1e-2, 1e-1};
        size_t z = 0;
        expect(invaskit_factor_workspace_bytes(&pb, &o, 3, &z) == INVASKIT_OK,
               "workspace of a grouped sweep", depth);
        invaskit_handle hs[3] = {nullptr, nullptr, nullptr};
        void* fake = reinterpret_cast<void*>(uintptr_t(1) << 30);
        expect(invaskit_factor_sweep(&pb, lam, 3, &o, fake, z - 256, nullptr, hs) ==
                   INVASKIT_E_WORKSPACE, "short sweep workspace", depth);
        const int st = invaskit_factor_sweep(&pb, lam, 3, &o, fake, z, nullptr, hs);
        expect(st != INVASKIT_OK && st != INVASKIT_E_ARG && st != INVASKIT_E_WORKSPACE &&
                   hs[0] == nullptr, "sweep device check", depth);
      }
      if (depth >= 1) {
        // malformed inputs: each refused with E_ARG
        Tree bad = t;
        bad.si[bad.so[1]] = (int32_t)(t.n + 5);  // outside every child skeleton
        invaskit_problem pbb = problem_of(bad);
        size_t b = 0;
        expect(invaskit_factor_workspace_bytes(&pbb, nullptr, 0, &b) == INVASKIT_E_ARG,
               "non-nested skeleton", depth);
        bad = t;
        bad.po[2] += 1;
        pbb = problem_of(bad);
        expect(invaskit_factor_workspace_bytes(&pbb, nullptr, 0, &b) == INVASKIT_E_ARG,
               "wrong P size", depth);
        bad = t;
        bad.leaf[1] = bad.leaf[0];
        pbb = problem_of(bad);
        expect(invaskit_factor_workspace_bytes(&pbb, nullptr, 0, &b) == INVASKIT_E_ARG,
               "empty leaf", depth);
      }
    }
  }
  // building blocks: workspace queries only
  {
    std::vector<int32_t> n = {1, 64, 65, 300, 1024};
    std::vector<int64_t> off(n.size(), 0);
    for (size_t i = 1; i < n.size(); ++i) off[i] = off[i - 1] + (int64_t)n[i - 1] * n[i - 1];
    std::vector<int32_t> nr = {1, 17, 33, 0, 4};
    std::vector<int64_t> ld(n.begin(), n.end()), boff(n.size(), 0);
    for (size_t i = 1; i < n.size(); ++i) boff[i] = boff[i - 1] + ld[i - 1] * nr[i - 1];
    void* fake = reinterpret_cast<void*>(uintptr_t(1) << 30);
    size_t need = 0;
    expect(invaskit_getrf_batched(INVASKIT_F32, fake, off.data(), n.data(), (int)n.size(),
                                  static_cast<int32_t*>(fake), static_cast<int32_t*>(fake),
                                  nullptr, 0, &need, nullptr) == INVASKIT_OK && need > 0,
           "getrf workspace query", 0);
    expect(invaskit_getrs_batched(INVASKIT_F64, fake, off.data(), n.data(),
                                  static_cast<int32_t*>(fake), fake, boff.data(), nr.data(),
                                  ld.data(), (int)n.size(), nullptr, 0, &need,
                                  nullptr) == INVASKIT_OK && need > 0,
           "getrs workspace query", 0);
  }
  std::printf("planning driver: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
