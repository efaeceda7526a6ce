"""Benchmark: INV-ASKIT factor + solve of lambda*I + K~ on one MI355X.

One step = refactor (every factorization phase: leaf blocks and LU, skeleton
blocks, leaf solves, projections, skeleton sweep, reduced systems and their
LU) + solve of the right-hand sides to relative residual <= 1e-10, checked
with the FP64 hierarchical product (both precisions verify it; FP64 refines
with its own factors if its direct solve misses).  The headline `value` is
the mixed-precision path (FP32 factors, FP64 top-level reduced systems, FP64
refinement); the plain FP64 path is timed on the same inputs beside it, and
its unverified direct solve alone for reference.  Each path also reports the
wall time of its first factorization from nothing (workspace query and
allocation, host planning, tile trials, factorization), cold and with the
tuning table warm.

Workload (default): N = 1,048,576 points in d = 8 from a 16-component unit
Gaussian mixture, depth-12 ball tree with uneven leaves of 64..512 points,
adaptive skeleton ranks (ID tolerance 1e-5, clamped to 32..256; the line
states the realized range), h = 0.5, lambda = 1e-4, one right-hand side.
All inputs are seeded and synthetic and resident in HBM before the timed
region.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--nrhs 1]

`--workload NAME` times one of the other synthetic workloads instead
(susy-wide: the same points with ranks spread over 32..256; tiny: N = 4,096
d = 8; covtype: N = 65,536 d = 54; mnist: N = 262,144 d = 784 sparse; normal:
N = 4,194,304 d = 64), under a metric line of its own; the headline line is
always the default workload.  `--sweep G` times a lambda sweep instead:
`--sweep-mode batched` factors all G lambdas in one sweep (launches batched
over --sweep-group lambdas) against G independent factorizations;
`--sweep-mode refactor` refactors one sweep handle per lambda (the 4M-point
workload holds one lambda at a time).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor+solve sec, FP32+refine vs FP64, N=1M d=8, rel residual ≤1e-10"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- HBM traffic
# Measured HBM bytes per launch come from two rocprofv3 counter runs of this
# script (FETCH_SIZE, then WRITE_SIZE), scaled by what the same counters read
# for a plain copy of known size in the same run (the FP64 copy of the
# right-hand side, N * nrhs * 8 bytes each way).  They are stored with the
# digest of the kernel's sources and reported only while that digest holds.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_susy_1m.json")
CSRC = os.path.join(ROOT, "paper_1602_01376_amd", "csrc")
COPY_KERNEL = "k_copy_cols<double, double>"
# phases whose time is one launch of a uniquely named kernel: name pattern
# (t = element type) and the source file that holds it
# the phase's kernel; {p} and {w} are its tile parameters (LU panel width and
# waves per matrix, or 16-column tiles per workgroup of the solves)
PHASE_KERNEL = {
    "leaf_lu_large": (r"k_getrf<{t}, {p}, \d+, 0, {w}, (?:true|false)>", "kernels_lu.hip"),
    "leaf_solves_large": (r"k_getrs<{t}, {t}, 0, {p}>", "kernels_trsm.hip"),
}
# leaves of at most this order form the library's small class (FP32, FP64),
# factored and solved on its second stream
SMALL_LEAF = {4: 192, 8: 256}


def phase_tile_params(phase, tiles):
    if phase == "leaf_lu_large":
        return dict(p=str(tiles["leaf_lu_panel"]), w=str(tiles["leaf_lu_waves"]))
    return dict(p=str(tiles["leaf_trsm_cols"] // 16), w="")


def source_digest(src):
    h = hashlib.sha256()
    for f in (src, "internal.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_kernel_name(name):
    name = re.sub(r"^void ", "", name)
    name = name.replace("invaskit::(anonymous namespace)::", "").replace("invaskit::", "")
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def read_counter_csv(path, counter):
    """Counter values per (kernel, grid size): the two leaf size classes
    launch the same kernel with different grids."""
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            key = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size"]))
            per.setdefault(key, []).append(float(r["Counter_Value"]))
    return per


def _by_name(per, name):
    return [v for (k, _), vals in per.items() if k == name for v in vals]


def write_traffic(fetch_csv, write_csv, copy_bytes, command):
    fetch = read_counter_csv(fetch_csv, "FETCH_SIZE")
    write = read_counter_csv(write_csv, "WRITE_SIZE")
    kib = copy_bytes / 1024.0
    copy_f, copy_w = np.mean(_by_name(fetch, COPY_KERNEL)), np.mean(_by_name(write, COPY_KERNEL))
    f_scale, w_scale = kib / copy_f, kib / copy_w
    entries = {}
    for phase, (pat, src) in PHASE_KERNEL.items():
        for t in ("float", "double"):
            rx = re.compile(pat.format(t=t, p=r"\d+", w=r"\d+") + "$")
            for (k, grid), vals in fetch.items():
                if not rx.match(k):
                    continue
                fk = float(np.mean(vals))
                wk = float(np.mean(write.get((k, grid), [0.0])))
                entries[f"{k} grid {grid}"] = {
                    "kernel": k, "grid": grid, "phase": phase, "dispatches": len(vals),
                    "fetch_kib": fk, "write_kib": wk,
                    "bytes": float((fk * f_scale + wk * w_scale) * 1024.0),
                    "source": src, "sha256": source_digest(src)}
    out = {"command": command, "calibration": {
        "kernel": COPY_KERNEL, "bytes_each_way": copy_bytes,
        "fetch_kib": float(copy_f), "write_kib": float(copy_w),
        "fetch_scale": float(f_scale), "write_scale": float(w_scale)}, "kernels": entries}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def traffic_for(phase, t, tiles):
    """Scaled HBM bytes per launch of the phase's kernel (the tile variant
    the factorization used), or None when no counters were taken for it or
    the kernel's sources changed since.  Of that kernel's launch grids the
    largest-traffic one is the large leaf class's launch (the small class
    and the tuner's trials on small sizes move fewer bytes)."""
    if phase not in PHASE_KERNEL or not os.path.exists(TRAFFIC_FILE):
        return None
    pat, src = PHASE_KERNEL[phase]
    rx = re.compile(pat.format(t=t, **phase_tile_params(phase, tiles)) + "$")
    with open(TRAFFIC_FILE) as fh:
        data = json.load(fh)
    digest = source_digest(src)
    found = [e["bytes"] for e in data.get("kernels", {}).values()
             if rx.match(e.get("kernel", "")) and e.get("sha256") == digest]
    return max(found) if found else None


# ----------------------------------------------------------- work accounting
def tree_sizes(pb):
    L = pb.depth
    nn = pb.n_nodes
    s = np.diff(pb.skel_offsets).astype(np.int64)
    size = np.zeros(nn, np.int64)
    for c in range(nn):
        a, b = pb.node_range(c)
        size[c] = b - a
    sib = lambda c: c + 1 if c & 1 else c - 1
    w = np.zeros(nn, np.int64)
    for c in range(1, nn):
        w[c] = s[sib(c)]
    return L, nn, s, size, w


def algorithmic_work(pb, esize, sym_leaves=False):
    """Flops and bytes per factorization phase for the schedule the library
    runs (exact sizes of this tree).  esize = bytes per factor element.  The
    kernel blocks count 2 d flops per entry (their FP64 Gram products on the
    matrix cores) when d > 64; at d <= 64 they count bytes only.
    sym_leaves: the large leaves were factored without row exchanges in the
    symmetric form (LDL^T work, m^3 / 3 flops) instead of LU (2 m^3 / 3)."""
    gram = 2.0 * pb.d if pb.d > 64 else 0.0
    L, nn, s, size, w = tree_sizes(pb)
    first_leaf = (1 << L) - 1
    leaves = range(first_leaf, nn)

    def anc(node, k):
        j = int(np.floor(np.log2(node + 1)))
        return (1 << k) - 1 + ((node - ((1 << j) - 1)) >> (j - k))

    z = np.zeros(nn, np.int64)
    for c in range(first_leaf):
        z[c] = s[2 * c + 1] + s[2 * c + 2]
    W = {k: dict(flops=0.0, bytes=0.0, launches=0) for k in
         ("leaf_blocks", "leaf_lu", "leaf_diag_inverses", "skeleton_blocks", "leaf_solves",
          "leaf_projections", "skeleton_sweep", "reduced_systems", "leaf_lu_large",
          "leaf_solves_large")}
    small = SMALL_LEAF[esize]
    for lf in leaves:
        m = size[lf]
        W["leaf_blocks"]["bytes"] += m * m * esize
        W["leaf_blocks"]["flops"] += gram * m * m
        lu_flops = (1.0 if sym_leaves and m > small else 2.0) / 3.0 * m ** 3
        W["leaf_lu"]["flops"] += lu_flops
        W["leaf_lu"]["bytes"] += 2.0 * m * m * esize
        if m > small:
            W["leaf_lu_large"]["flops"] += lu_flops
            W["leaf_lu_large"]["bytes"] += 2.0 * m * m * esize
        nb = -(-m // 64)
        W["leaf_diag_inverses"]["flops"] += nb * 2.0 * 64 ** 3 / 3.0
        W["leaf_diag_inverses"]["bytes"] += nb * 3 * 64 * 64 * esize
    # one launch each, except the leaf LU, inverses and solves: one per size
    # class (the large class's own launches are the *_large entries)
    has_small = bool(np.any(size[first_leaf:] <= small))
    has_large = bool(np.any(size[first_leaf:] > small))
    W["leaf_blocks"]["launches"] = 1
    for key in ("leaf_lu", "leaf_diag_inverses"):
        W[key]["launches"] = int(has_small) + int(has_large)
    W["leaf_lu_large"]["launches"] = int(has_large)
    for k in range(L, 0, -1):
        for lf in leaves:
            m = size[lf]
            c = anc(lf, k)
            wk = w[c]
            W["skeleton_blocks"]["bytes"] += m * wk * esize
            W["skeleton_blocks"]["flops"] += gram * m * wk
            W["leaf_solves"]["flops"] += 2.0 * m * m * wk
            W["leaf_solves"]["bytes"] += 2 * m * wk * esize
            if m > small:
                W["leaf_solves_large"]["flops"] += 2.0 * m * m * wk
                W["leaf_solves_large"]["bytes"] += 2 * m * wk * esize
            W["leaf_projections"]["flops"] += 2.0 * s[lf] * m * wk
            W["leaf_projections"]["bytes"] += (s[lf] * m + m * wk + s[lf] * wk) * esize
        for j in range(L - 1, k - 1, -1):
            for bn in range((1 << j) - 1, (2 << j) - 1):
                wk = w[anc(bn, k)]
                W["skeleton_sweep"]["flops"] += 2.0 * z[bn] ** 2 * wk + 2.0 * s[bn] * z[bn] * wk
                W["skeleton_sweep"]["bytes"] += (s[bn] * z[bn] + 3 * z[bn] * wk) * esize
        for a in range((1 << (k - 1)) - 1, (1 << k) - 1):
            W["reduced_systems"]["flops"] += 2.0 / 3.0 * z[a] ** 3
            W["reduced_systems"]["bytes"] += 3.0 * z[a] ** 2 * esize
    # one launch each over every level's columns; the sweep and the reduced
    # systems run as one wavefront step (two launches) per level
    for key in ("skeleton_blocks", "leaf_projections"):
        W[key]["launches"] = 1
    W["leaf_solves"]["launches"] = int(has_small) + int(has_large)
    W["leaf_solves_large"]["launches"] = int(has_large) if L > 0 else 0
    # the reduced-system factor is read once per sweep step (all factor levels)
    for j in range(1, L):
        for bn in range((1 << j) - 1, (2 << j) - 1):
            W["skeleton_sweep"]["bytes"] += z[bn] ** 2 * esize
    W["skeleton_sweep"]["launches"] = 2 * max(L - 1, 0)
    W["reduced_systems"]["launches"] = 3 * L
    for lf in leaves:  # the leaf LU is read once by the all-level leaf solve
        W["leaf_solves"]["bytes"] += size[lf] ** 2 * esize
        if size[lf] > small:
            W["leaf_solves_large"]["bytes"] += size[lf] ** 2 * esize
    return W


def paper_literal_flops(pb):
    """Flops of Algorithms 1-2 as the oracle runs them (explicit full P,
    W = Solve(child, K block) through the whole subtree)."""
    L, nn, s, size, w = tree_sizes(pb)
    first_leaf = (1 << L) - 1
    z = np.zeros(nn, np.int64)
    for c in range(first_leaf):
        z[c] = s[2 * c + 1] + s[2 * c + 2]

    def solve_cost(node, r):
        if node >= first_leaf:
            return 2.0 * size[node] ** 2 * r
        l, rr = 2 * node + 1, 2 * node + 2
        return (solve_cost(l, r) + solve_cost(rr, r) + 4.0 * (s[rr] * size[rr] + s[l] * size[l]) * r
                + 2.0 * z[node] ** 2 * r)

    f = sum(2.0 / 3.0 * size[lf] ** 3 for lf in range(first_leaf, nn))
    for a in range(first_leaf):
        l, r = 2 * a + 1, 2 * a + 2
        f += solve_cost(l, s[r]) + solve_cost(r, s[l])
        f += 2.0 * (s[r] * size[r] * s[l] + s[l] * size[l] * s[r]) + 2.0 / 3.0 * z[a] ** 3
        if a > 0:
            f += 2.0 * s[a] * (s[l] * size[l] + s[r] * size[r])
    return f + solve_cost(0, 1)


# --------------------------------------------------------------- CPU baseline
def cpu_baseline(full_pb, samples=((32768, 7), (65536, 8))):
    """The FP64 oracle (Algorithms 1-2 with NumPy/SciPy LAPACK, untuned) timed
    on the host cores on bounded samples of the same generator, each scaled
    to the full workload by the paper-literal flop ratio; the two samples'
    estimates check that scaling law."""
    import oracle
    from paper_1602_01376_amd.setup import make_problem, rhs_for
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        cores = os.cpu_count() or 1
    name = full_pb.name if full_pb.name else "susy"
    runs = []
    for n, depth in samples:
        pb = make_problem(name, n=n, depth=depth)
        b = rhs_for(pb, nrhs=1)
        t0 = time.perf_counter()
        F = oracle.factorize(pb, pb.lam)
        oracle.solve(F, b)
        t = time.perf_counter() - t0
        ratio = paper_literal_flops(full_pb) / paper_literal_flops(pb)
        runs.append(dict(n=n, depth=depth, seconds=t, flop_ratio=ratio, estimate_s=t * ratio))
        log(f"cpu baseline sample N={n}: {t:.2f} s, estimate {t * ratio:.1f} s")
    est = runs[-1]["estimate_s"]
    return {"value": est, "unit": "s", "cores": int(cores), "kind": "oracle",
            "sample": (f"FP64 oracle factor+solve (Algorithms 1-2, NumPy/SciPy LAPACK) on the same "
                       f"generator at N={runs[-1]['n']} (depth {runs[-1]['depth']}): "
                       f"{runs[-1]['seconds']:.2f} s, scaled by the paper-literal flop ratio "
                       f"{runs[-1]['flop_ratio']:.1f}; the N={runs[0]['n']} sample scales to "
                       f"{runs[0]['estimate_s']:.0f} s"),
            "samples": runs,
            "scaling_check": runs[0]["estimate_s"] / runs[-1]["estimate_s"]}


def rank_summary(pb):
    ranks = np.diff(pb.skel_offsets)[1:]
    sizes = np.diff(pb.leaf_offsets)
    return dict(leaf_min=int(sizes.min()), leaf_max=int(sizes.max()), rank_min=int(ranks.min()),
                rank_max=int(ranks.max()), rank_median=float(np.median(ranks)),
                at_floor=float(np.mean(ranks == ranks.min())))


def power_estimate(apply, n, iters, seed=5):
    """|largest eigenvalue| of a linear map by power iteration."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    x /= x.norm()
    lam = 0.0
    for _ in range(iters):
        y = apply(x)
        lam = float(y.norm())
        x = y / lam
    return lam


def kappa_estimate(fac, n, iters=25):
    """kappa(lambda I + K~) estimated as rho(A) rho(A^-1), both by power
    iteration with the library's FP64 product and solve (a lower estimate of
    the 2-norm condition number for this nearly symmetric matrix)."""
    rho = power_estimate(lambda v: fac.matvec(v), n, iters)
    rinv = power_estimate(lambda v: fac.solve(v, check=False), n, iters)
    return dict(rho_A=rho, rho_Ainv=rinv, kappa=rho * rinv, iterations=iters)


# ----------------------------------------------------------------------- main
def time_first_factor(binding, pb, lam, mode, X, P, kw):
    """Wall time of a Factorization from nothing: workspace query, workspace
    allocation (PyTorch), host planning, table upload and the factorization
    (tile trials included when the tuning table misses)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = binding.Factorization(pb, lam, precision=mode, points=X, p_values=P, **kw)
    torch.cuda.synchronize()
    return fac, time.perf_counter() - t0


def run_sweep(args, binding, pb, X, P, b):
    import torch
    lams = list(np.logspace(-6, -1, args.sweep))
    kw = dict(precision=args.sweep_precision, points=X, p_values=P,
              fp64_top_levels=args.fp64_top_levels)
    per = []
    if args.sweep_mode == "batched":
        # every lambda in one sweep workspace, batched launches of
        # --sweep-group lambdas (0: all)
        # warm-up of both forms: kernel loads, tile trials of the batched
        # and of the single launches, and PyTorch's cached blocks
        for f in binding.factor_sweep(pb, lams, lambda_group=args.sweep_group, **kw):
            f.close()
        fac = binding.Factorization(pb, lams[0], **kw)
        fac.close()
        del fac
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        facs = binding.factor_sweep(pb, lams, lambda_group=args.sweep_group, **kw)
        torch.cuda.synchronize()
        t_sweep = time.perf_counter() - t0
        for lam, f in zip(lams, facs):
            t1 = time.perf_counter()
            _, info, st = f.solve(b, return_info=True, check=False)
            torch.cuda.synchronize()
            per.append(dict(lam=lam, solve_s=time.perf_counter() - t1, status=st, **info))
        ws = facs[0]._ws.numel()
        phase = facs[0].phase_times()
        for f in facs:
            f.close()
        del facs
        t0 = time.perf_counter()
        for lam in lams:
            f = binding.Factorization(pb, lam, **kw)
            f.close()
            del f
        torch.cuda.synchronize()
        t_sep = time.perf_counter() - t0
        out = dict(sweep_s=t_sweep, separate_s=t_sep, sweep_phase_ms=phase,
                   per_lambda_sweep_ms=1e3 * t_sweep / len(lams),
                   per_lambda_separate_ms=1e3 * t_sep / len(lams))
    else:
        # one handle of a sweep (the lambda-free kernel blocks evaluated once
        # into its workspace), refactored for every lambda; each factor is
        # solved right away (the workload's memory holds one lambda at a time)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = binding.factor_sweep(pb, lams[:1], **kw)[0]
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        ws = f._ws.numel()
        log(f"sweep handle: workspace {ws / 1e9:.1f} GB, first factor {first:.2f} s")
        for i, lam in enumerate(lams):
            t1 = time.perf_counter()
            if i > 0:
                f.refactor(lam)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, info, st = f.solve(b, return_info=True, check=False)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            per.append(dict(lam=lam, factor_s=(t2 - t1) if i > 0 else first, solve_s=t3 - t2,
                            status=st, factor_phase_ms=f.phase_times(), **info))
            log(f"lambda {lam:.1e}: factor {per[-1]['factor_s']:.3f} s, solve {t3 - t2:.3f} s, "
                f"residual {info['final_rel_residual']:.2e} ({info['iterations']} steps)")
        f.close()
        out = dict(first_factor_s=first,
                   per_lambda_refactor_ms=1e3 * float(np.mean([p["factor_s"] for p in per[1:]]))
                   if len(per) > 1 else None)
    print(json.dumps({"metric": "lambda-sweep factorization seconds", "lambdas": lams,
                      "workload": args.workload, "n": pb.n, "d": pb.d, "mode": args.sweep_mode,
                      "sweep_group": args.sweep_group, "nrhs": args.nrhs,
                      "precision": args.sweep_precision, "workspace_gb": ws / 1e9,
                      "per_lambda": per,
                      "per_lambda_solve_ms": 1e3 * float(np.mean([p["solve_s"] for p in per])),
                      "max_refined_residual": max(p["final_rel_residual"] for p in per),
                      **out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides (default: 1 for the headline, else the workload's)")
    ap.add_argument("--workload", default="susy",
                    choices=["susy", "susy-wide", "tiny", "covtype", "mnist", "normal"],
                    help="synthetic workload (default susy: the headline configuration)")
    ap.add_argument("--n", type=int, default=None, help="scale the workload down (testing)")
    ap.add_argument("--depth", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kappa", action="store_true",
                    help="skip the power-iteration condition estimate")
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--fp64-top-levels", type=int, default=4,
                    help="mixed precision: reduced systems of the levels above this are FP64")
    ap.add_argument("--tune", choices=["auto", "off"], default="auto",
                    help="tile autotuning of the leaf LU and leaf solves")
    ap.add_argument("--lu-panel", type=int, default=0, choices=[0, 16, 32],
                    help="fix the leaf LU panel width (0: per --tune)")
    ap.add_argument("--lu-waves", type=int, default=0, choices=[0, 4, 8],
                    help="fix the leaf LU's waves per matrix (0: per --tune)")
    ap.add_argument("--trsm-cols", type=int, default=0, choices=[0, 16, 32],
                    help="fix the leaf solves' right-hand sides per workgroup (0: per --tune)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic record from two rocprofv3 counter runs of "
                         "this script (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--traffic-command", default="", help="the counter command, recorded")
    ap.add_argument("--sweep", type=int, default=0, metavar="G",
                    help="instead of the headline step: factor G lambdas (logspace(-6, -1, G)) "
                         "sharing one evaluation of the kernel blocks, and solve each")
    ap.add_argument("--sweep-mode", choices=["batched", "refactor"], default="batched",
                    help="batched: all G handles of one sweep, launches batched over "
                         "--sweep-group lambdas, timed against G independent factorizations; "
                         "refactor: one sweep handle refactored for each lambda (for workloads "
                         "whose memory holds one lambda at a time)")
    ap.add_argument("--sweep-group", type=int, default=0, metavar="S",
                    help="with --sweep-mode batched: lambdas per batched launch (0: all)")
    ap.add_argument("--sweep-precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--lam", type=float, default=None, help="override the workload's lambda")
    args = ap.parse_args()
    headline = args.workload == "susy"
    if args.nrhs is None:
        from paper_1602_01376_amd.setup.problem import WORKLOADS
        args.nrhs = 1 if headline else WORKLOADS[args.workload]["nrhs"]
    if args.traffic_from:
        n = args.n or (1 << 20)
        out = write_traffic(*args.traffic_from, copy_bytes=8 * n * args.nrhs,
                            command=args.traffic_command)
        print(json.dumps(out, indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the multi-GPU sharding of the tree is a design "
              "note, not part of this build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1602_01376_amd import binding
    from paper_1602_01376_amd.setup import make_problem, rhs_for

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    pb = make_problem(args.workload, n=args.n, depth=args.depth,
                      progress=lambda text: log(f"setup: {text}"))
    rs = rank_summary(pb)
    log(f"setup {time.perf_counter() - t0:.1f} s: N={pb.n} d={pb.d} L={pb.depth} {rs}")
    X = torch.from_numpy(pb.X).cuda()
    P = torch.from_numpy(pb.p_values).cuda()
    b = torch.from_numpy(rhs_for(pb, nrhs=args.nrhs)).cuda()
    if args.lam is not None:
        pb.lam = args.lam
    lam = pb.lam

    if args.sweep > 0:
        run_sweep(args, binding, pb, X, P, b)
        return

    results = {}
    kappa = None
    modes = ["mixed", "fp64"] if args.only == "both" else [args.only]
    for mode in modes:
        kw = dict(tune=args.tune, leaf_lu_panel=args.lu_panel, leaf_trsm_cols=args.trsm_cols,
                  leaf_lu_waves=args.lu_waves, fp64_top_levels=args.fp64_top_levels)
        fac, first = time_first_factor(binding, pb, lam, mode, X, P, kw)
        tiles = fac.tile_config()  # the first factor's trials, if it tuned
        # a second handle from nothing, the tuning table now warm
        fac2, first_warm = time_first_factor(binding, pb, lam, mode, X, P, kw)
        plan_ms = fac2.phase_times()["handle_planning"]
        fac2.close()
        del fac2
        log(f"{mode}: workspace {fac.device_bytes() / 2**30:.2f} GiB, first factor {first:.3f} s "
            f"(tuning table warm: {first_warm:.3f} s, planning {plan_ms:.1f} ms), tiles {tiles}")
        for _ in range(args.warmup):
            fac.refactor(lam)
            fac.solve(b, return_info=True, check=False)
        phases = {}
        tf = ts = 0.0
        info = None
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            a = time.perf_counter()
            fac.refactor(lam)       # synchronizes at its end (pivot status)
            bpt = time.perf_counter()
            x, info, st = fac.solve(b, return_info=True, check=False)
            torch.cuda.synchronize()
            c = time.perf_counter()
            tf += bpt - a
            ts += c - bpt
            for k, v in fac.phase_times().items():
                phases[k] = phases.get(k, 0.0) + v
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_start) / args.steps
        results[mode] = dict(
            seconds=wall, factor_s=tf / args.steps, solve_s=ts / args.steps,
            final_rel_residual=info["final_rel_residual"],
            unrefined_rel_residual=info["unrefined_rel_residual"],
            iterations=info["iterations"], gmres_iterations=info["gmres_iterations"],
            method=info["method"], converged=bool(info["converged"]), status=st,
            first_factor_s=first, first_factor_warm_s=first_warm, planning_ms=plan_ms,
            phase_ms={k: v / args.steps for k, v in phases.items()},
            workspace_gib=fac.device_bytes() / 2**30, tiles=tiles)
        if mode == "fp64" and not args.no_kappa:
            kappa = kappa_estimate(fac, pb.n)
            log(f"kappa estimate {kappa}")
        fac.close()
        del fac
        if mode == "fp64":
            # the direct solve alone (refine = none, no residual check), for
            # reference: the headline FP64 time above verifies the residual
            facn = binding.Factorization(pb, lam, precision="fp64", points=X, p_values=P,
                                         refine="none", **kw)
            facn.solve(b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                facn.solve(b)
            torch.cuda.synchronize()
            results[mode]["direct_solve_s"] = (time.perf_counter() - t1) / args.steps
            facn.close()
            del facn
        log(mode, json.dumps(results[mode]))
        torch.cuda.empty_cache()

    head = results.get("mixed") or results["fp64"]
    esize = 4 if "mixed" in results else 8
    dtype = "f32" if "mixed" in results else "f64"
    ctype = "float" if dtype == "f32" else "double"
    work = algorithmic_work(pb, esize, sym_leaves=head["tiles"].get("leaf_pivoting") == 0)
    # dominant kernel: the single-launch phase with the largest measured time
    ph = head["phase_ms"]
    cand = {k: ph.get(k, 0.0) for k in work if work[k]["launches"] == 1}
    dom = max(cand, key=cand.get)
    wk = work[dom]
    per_launch_ms = ph[dom] / max(wk["launches"], 1)
    traffic = (traffic_for(dom, ctype, head["tiles"])
               if (headline and args.n is None and args.nrhs == 1) else None)
    if wk["flops"] > 0:
        achieved = wk["flops"] / wk["launches"] / (per_launch_ms * 1e-3) / 1e12
        # the kernel blocks' Gram products run in FP64 in both precisions
        peak = PEAK_TFLOPS["f64" if dom in ("leaf_blocks", "skeleton_blocks") else dtype]
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": dom, "launches": wk["launches"], "avg_launch_ms": per_launch_ms,
                "algorithmic_tflop": wk["flops"] / 1e12, "algorithmic_gb": wk["bytes"] / 1e9}
    else:
        achieved = wk["bytes"] / wk["launches"] / (per_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "launches": wk["launches"], "avg_launch_ms": per_launch_ms,
                "algorithmic_gb": wk["bytes"] / 1e9}
    ranks = (f"leaves {rs['leaf_min']}..{rs['leaf_max']}, adaptive ranks (ID tolerance "
             f"{'1e-5' if headline else 'per workload'}) realized {rs['rank_min']}..{rs['rank_max']}, "
             f"median {rs['rank_median']:.0f}, {100 * rs['at_floor']:.1f}% at the floor")
    out = {
        "metric": METRIC if headline else (
            f"factor+solve sec, FP32+refine vs FP64, {args.workload} N={pb.n} d={pb.d}, "
            "rel residual ≤1e-10"),
        "value": head["seconds"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["seconds"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if "mixed" in results else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: gaussian-mixture N={pb.n} d={pb.d}, ball tree "
                                f"depth {pb.depth}, {ranks}, h={pb.h}, lambda={lam}"),
                   "nrhs": args.nrhs, "precision": "mixed" if "mixed" in results else "fp64",
                   "fp64_top_levels": args.fp64_top_levels},
        "roofline": roof,
        "paths": results,
        "work_tflop": {k: v["flops"] / 1e12 for k, v in work.items()},
        "kappa_estimate": kappa,
    }
    if "mixed" in results:
        out["first_factor_s"] = results["mixed"]["first_factor_s"]
        out["first_factor_warm_s"] = results["mixed"]["first_factor_warm_s"]
    if "mixed" in results and "fp64" in results:
        out["speedup_vs_fp64"] = results["fp64"]["seconds"] / results["mixed"]["seconds"]
    if not args.no_cpu_baseline and headline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(pb)
        log(f"cpu baseline {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
