"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid input before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "invaskit.h")
LIB = os.path.join(ROOT, "paper_1602_01376_amd", "libinvaskit.so")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(invaskit_\w+)\s*\(", txt, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("invaskit_factor", "invaskit_solve", "invaskit_matvec", "invaskit_destroy",
              "invaskit_refactor", "invaskit_getrf_batched", "invaskit_getrs_batched",
              "invaskit_kernel_blocks", "invaskit_status_string", "invaskit_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1602_01376_amd import binding
    assert sorted(binding.EXPORTED) == _declared()


def test_status_strings():
    from paper_1602_01376_amd import binding
    lib = binding.library()
    assert lib.invaskit_status_string(0) == b"ok"
    assert lib.invaskit_status_string(-4) == b"singular pivot"
    assert lib.invaskit_status_string(-99) == b"unknown status"


def _raw_problem(pb, **over):
    from paper_1602_01376_amd import binding
    arrs = dict(leaf=np.ascontiguousarray(pb.leaf_offsets, np.int64),
                so=np.ascontiguousarray(pb.skel_offsets, np.int64),
                si=np.ascontiguousarray(pb.skel_index, np.int32),
                po=np.ascontiguousarray(pb.p_offsets, np.int64))
    arrs.update({k: v for k, v in over.items() if k in arrs})
    fields = dict(n=pb.n, d=pb.d, depth=pb.depth, points_dtype=0, reserved0=0,
                  points=0x1000, leaf_offsets=arrs["leaf"].ctypes.data,
                  skel_offsets=arrs["so"].ctypes.data, skel_index=arrs["si"].ctypes.data,
                  p_offsets=arrs["po"].ctypes.data, p_values=0x2000, h=pb.h)
    fields.update({k: v for k, v in over.items() if k not in arrs})
    return binding._Problem(**fields), arrs


@pytest.fixture(scope="module")
def small_problem():
    from paper_1602_01376_amd.setup import make_problem
    return make_problem("tiny", n=512, depth=2)


def _factor_status(raw, lam=1e-2, opt=None, ws=None, ws_bytes=0):
    from paper_1602_01376_amd import binding
    h = C.c_void_p()
    st = binding.library().invaskit_factor(C.byref(raw), lam, C.byref(opt) if opt else None,
                                           ws, ws_bytes, None, C.byref(h))
    return st, binding.last_error()


@pytest.mark.parametrize("case,expect", [
    (dict(n=0), "n must be"),
    (dict(d=0), "d must be"),
    (dict(depth=-1), "depth"),
    (dict(points_dtype=7), "points_dtype"),
    (dict(points=0), "points is NULL"),
    (dict(h=-1.0), "h must be"),
    (dict(h=float("nan")), "h must be"),
])
def test_invalid_scalars_rejected(small_problem, case, expect):
    raw, keep = _raw_problem(small_problem, **case)
    st, msg = _factor_status(raw)
    assert st == -1 and expect in msg


def test_bad_offsets_rejected(small_problem):
    leaf = np.array(small_problem.leaf_offsets, np.int64)
    leaf[-1] += 1
    raw, keep = _raw_problem(small_problem, leaf=leaf)
    st, msg = _factor_status(raw)
    assert st == -1 and "end at n" in msg
    leaf = np.array(small_problem.leaf_offsets, np.int64)
    leaf[2] = leaf[1]
    raw, keep = _raw_problem(small_problem, leaf=leaf)
    st, msg = _factor_status(raw)
    assert st == -1 and "points" in msg


def test_non_nested_skeleton_rejected(small_problem):
    si = np.array(small_problem.skel_index, np.int32)
    so = small_problem.skel_offsets
    si[so[1]] = 10**6  # node 1 (internal) gets a point that is in no child skeleton
    raw, keep = _raw_problem(small_problem, si=si)
    st, msg = _factor_status(raw)
    assert st == -1 and "not nested" in msg


def test_leaf_skeleton_outside_leaf_rejected(small_problem):
    si = np.array(small_problem.skel_index, np.int32)
    so = small_problem.skel_offsets
    leaf_node = 3
    si[so[leaf_node]] = small_problem.n - 1  # belongs to the last leaf
    raw, keep = _raw_problem(small_problem, si=si)
    st, msg = _factor_status(raw)
    assert st == -1 and "leaves the leaf" in msg


def test_wrong_p_size_rejected(small_problem):
    po = np.array(small_problem.p_offsets, np.int64)
    po[2:] += 1
    raw, keep = _raw_problem(small_problem, po=po)
    st, msg = _factor_status(raw)
    assert st == -1 and "P of node" in msg


def test_bad_options_rejected(small_problem):
    from paper_1602_01376_amd import binding
    raw, keep = _raw_problem(small_problem)
    opt = binding._Options()
    binding.library().invaskit_default_options(C.byref(opt))
    assert opt.precision == 0 and opt.fp64_top_levels == 4 and opt.refine_tol == 1e-10
    opt.precision = 5
    st, msg = _factor_status(raw, opt=opt)
    assert st == -1 and "precision" in msg
    binding.library().invaskit_default_options(C.byref(opt))
    opt.max_refine_iters = 0
    st, msg = _factor_status(raw, opt=opt)
    assert st == -1
    binding.library().invaskit_default_options(C.byref(opt))
    assert opt.tune == binding.TUNE_AUTO and opt.leaf_lu_panel == 0 and opt.leaf_trsm_cols == 0
    assert opt.leaf_lu_waves == 0
    opt.tune = 7
    st, msg = _factor_status(raw, opt=opt)
    assert st == -1 and "tune" in msg
    for field, v in (("leaf_lu_panel", 24), ("leaf_trsm_cols", 64), ("leaf_trsm_cols", -16)):
        binding.library().invaskit_default_options(C.byref(opt))
        setattr(opt, field, v)
        st, msg = _factor_status(raw, opt=opt)
        assert st == -1 and "leaf_lu_panel and leaf_trsm_cols" in msg, (field, v)
    for v in (2, 16, -4):
        binding.library().invaskit_default_options(C.byref(opt))
        opt.leaf_lu_waves = v
        st, msg = _factor_status(raw, opt=opt)
        assert st == -1 and "leaf_lu_waves" in msg, v
    binding.library().invaskit_default_options(C.byref(opt))
    assert opt.refine == binding.REFINE["auto"] and opt.gmres_restart == 20
    assert opt.max_gmres_iters == 300
    for field, v, word in (("refine", 4, "refine"), ("refine", -1, "refine"),
                           ("gmres_restart", 1, "gmres_restart"),
                           ("gmres_restart", 65, "gmres_restart"),
                           ("max_gmres_iters", 0, "max_gmres_iters"),
                           ("zlu_form", 3, "zlu_form"), ("zlu_form", -1, "zlu_form"),
                           ("zsolve_cols", 24, "zsolve_cols"),
                           ("leaf_pivoting", 2, "leaf_pivoting")):
        binding.library().invaskit_default_options(C.byref(opt))
        setattr(opt, field, v)
        st, msg = _factor_status(raw, opt=opt)
        assert st == -1 and word in msg, (field, v)


def test_options_struct_layout():
    """The binding's mirrors of invaskit_options and invaskit_solve_info have
    the header's sizes and field offsets (options: 4 + 4 + 8 + 12 x 4 bytes)."""
    from paper_1602_01376_amd import binding
    O = binding._Options
    assert C.sizeof(O) == 64
    assert O.refine_tol.offset == 8 and O.max_refine_iters.offset == 16
    assert O.tune.offset == 20 and O.leaf_lu_panel.offset == 24
    assert O.leaf_trsm_cols.offset == 28 and O.leaf_lu_waves.offset == 32
    assert O.refine.offset == 36 and O.gmres_restart.offset == 40
    assert O.max_gmres_iters.offset == 44 and O.lambda_group.offset == 48
    assert O.zlu_form.offset == 52 and O.zsolve_cols.offset == 56
    assert O.leaf_pivoting.offset == 60
    S = binding.SolveInfo
    assert C.sizeof(S) == 32 and S.final_rel_residual.offset == 8
    assert S.gmres_iterations.offset == 24 and S.method.offset == 28
    T = binding._TileConfig
    assert C.sizeof(T) == 64 and T.lu_ms.offset == 16 and T.trsm_ms.offset == 32
    assert T.leaf_trsm_cols_small.offset == 40 and T.trsm_small_ms.offset == 44
    assert T.zlu_one_wave_levels.offset == 52 and T.zsolve32_levels.offset == 56
    assert T.leaf_pivoting.offset == 60


def test_tuning_table_text_round_trip():
    """Export, import and clear of the process-wide tuning table (host only);
    a malformed import changes nothing."""
    from paper_1602_01376_amd import binding
    binding.tuning_clear()
    assert binding.tuning_table() == {}
    entries = {"getrf.f32.n512.c24.w67": 16, "getrfw.f32.n512.c24.w67": 8,
               "getrs.f64.k0.n256.w60": 32, "zgetrf.f32.n142.c20": 1,
               "zgetrf.f64.n128.c0": 2, "getrs.f32.k1.n142.w50": 16}
    binding.tuning_load(entries)
    assert binding.tuning_table() == entries
    lib = binding.library()
    for bad in (b"getrf.f32.n1 24\n", b"getrs.f32 16 extra\n", b"other.key 16\n",
                b"getrf.f32.n1\n", b"getrfw.f32.n1 16\n", b"getrf.f32.n1 8\n",
                b"zgetrf.f32.n1 16\n", b"zgetrf.f32.n1 0\n"):
        assert lib.invaskit_tuning_import(bad) == -1, bad
    assert binding.tuning_table() == entries
    need = C.c_size_t()
    assert lib.invaskit_tuning_export(None, 0, C.byref(need)) == 0
    full = "".join(f"{k} {v}\n" for k, v in sorted(entries.items()))
    assert need.value == len(full) + 1
    small = C.create_string_buffer(8)
    assert lib.invaskit_tuning_export(small, 8, C.byref(need)) == 0
    assert small.value == full[:7].encode()
    assert lib.invaskit_tuning_export(None, 0, None) == -1
    binding.tuning_clear()
    assert binding.tuning_table() == {}


def test_nonfinite_lambda_rejected(small_problem):
    raw, keep = _raw_problem(small_problem)
    st, msg = _factor_status(raw, lam=float("inf"))
    assert st == -1 and "lambda" in msg


def test_sweep_arguments_rejected(small_problem):
    """invaskit_factor_sweep validates every lambda and its arrays before any
    device work; out entries stay NULL."""
    from paper_1602_01376_amd import binding
    lib = binding.library()
    raw, keep = _raw_problem(small_problem)
    out = (C.c_void_p * 3)()
    lams = (C.c_double * 3)(1e-2, float("inf"), 1e-1)
    assert lib.invaskit_factor_sweep(C.byref(raw), lams, 3, None, None, 0, None, out) == -1
    assert "lambda" in binding.last_error()
    assert all(v is None for v in out)
    assert lib.invaskit_factor_sweep(C.byref(raw), lams, 0, None, None, 0, None, out) == -1
    assert lib.invaskit_factor_sweep(C.byref(raw), None, 3, None, None, 0, None, out) == -1
    bad, keep2 = _raw_problem(small_problem, d=0)
    ok = (C.c_double * 2)(1e-2, 1e-1)
    assert lib.invaskit_factor_sweep(C.byref(bad), ok, 2, None, None, 0, None, out) == -1


def test_null_handle_calls_are_rejected():
    from paper_1602_01376_amd import binding
    lib = binding.library()
    assert lib.invaskit_solve(None, None, 1, 1, None, 1, None, 0, None) == -1
    assert lib.invaskit_matvec(None, None, 1, 1, None, 1, None, 0) == -1
    need = C.c_size_t()
    assert lib.invaskit_solve_workspace_bytes(None, 1, C.byref(need), None) == -1
    assert lib.invaskit_matvec_workspace_bytes(None, 1, C.byref(need)) == -1
    assert lib.invaskit_refactor(None, 1.0) == -1
    assert lib.invaskit_destroy(None) == 0


def _ws_bytes(raw, n_lambda, precision=0, lambda_group=0):
    from paper_1602_01376_amd import binding
    opt = binding._Options()
    binding.library().invaskit_default_options(C.byref(opt))
    opt.precision = precision
    opt.lambda_group = lambda_group
    out = C.c_size_t()
    st = binding.library().invaskit_factor_workspace_bytes(C.byref(raw), C.byref(opt), n_lambda,
                                                           C.byref(out))
    assert st == 0, binding.last_error()
    return out.value, opt


def test_factor_workspace_sizes(small_problem):
    """Workspace queries are host-only (they run here, without a GPU): a
    sweep needs more than one factorization and grows with its lambdas;
    FP32 factors need less than FP64; lambda groups of one need no batched
    tables; and the size covers at least the leaf factors and W storage."""
    raw, keep = _raw_problem(small_problem)
    single, _ = _ws_bytes(raw, 0)
    one, _ = _ws_bytes(raw, 1)
    three, _ = _ws_bytes(raw, 3)
    three_g1, _ = _ws_bytes(raw, 3, lambda_group=1)
    mixed, _ = _ws_bytes(raw, 0, precision=1)
    assert single < one < three and three_g1 < three
    assert mixed < single
    m = np.diff(small_problem.leaf_offsets)
    assert single > 8 * int(np.sum(m * m))
    from paper_1602_01376_amd import binding
    out = C.c_size_t()
    assert binding.library().invaskit_factor_workspace_bytes(C.byref(raw), None, -1,
                                                             C.byref(out)) == -1
    bad, keep2 = _raw_problem(small_problem, d=0)
    assert binding.library().invaskit_factor_workspace_bytes(C.byref(bad), None, 0,
                                                             C.byref(out)) == -1


def test_small_or_misaligned_workspace_rejected_before_any_launch(small_problem):
    """A workspace one byte short fails with INVASKIT_E_WORKSPACE and a
    misaligned one with INVASKIT_E_ARG, both before the library looks for a
    device (the addresses here are placeholders that nothing dereferences);
    one of the full size passes those checks and only then needs the GPU."""
    from paper_1602_01376_amd import binding
    raw, keep = _raw_problem(small_problem)
    need, opt = _ws_bytes(raw, 0)
    fake = C.c_void_p(1 << 20)
    st, msg = _factor_status(raw, opt=opt, ws=fake, ws_bytes=need - 1)
    assert st == binding.E_WORKSPACE and str(need) in msg
    st, msg = _factor_status(raw, opt=opt, ws=C.c_void_p((1 << 20) + 8), ws_bytes=need)
    assert st == binding.E_ARG and "aligned" in msg
    st, msg = _factor_status(raw, opt=opt, ws=None, ws_bytes=need)
    assert st == binding.E_ARG and "NULL" in msg
    need3, opt3 = _ws_bytes(raw, 3)
    out = (C.c_void_p * 3)()
    lams = (C.c_double * 3)(1e-2, 1e-1, 1.0)
    st = binding.library().invaskit_factor_sweep(C.byref(raw), lams, 3, C.byref(opt3), fake,
                                                 need3 - 256, None, out)
    assert st == binding.E_WORKSPACE and all(v is None for v in out)


def test_building_block_workspace_queries():
    """With workspace = NULL a building block reports its workspace size and
    launches nothing (host only)."""
    from paper_1602_01376_amd import binding
    lib = binding.library()
    n = np.array([5, 70, 130], np.int32)
    offs = np.array([0, 25, 25 + 4900], np.int64)
    need = C.c_size_t()
    fake = C.c_void_p(1 << 20)
    assert lib.invaskit_getrf_batched(0, fake, binding._ptr(offs), binding._ptr(n), 3, fake, fake,
                                      None, 0, C.byref(need), None) == 0
    assert need.value >= 3 * 32
    nr = np.array([1, 16, 40], np.int32)
    ld = n.astype(np.int64)
    boffs = np.array([0, 5, 5 + 70 * 16], np.int64)
    assert lib.invaskit_getrs_batched(0, fake, binding._ptr(offs), binding._ptr(n), fake, fake,
                                      binding._ptr(boffs), binding._ptr(nr), binding._ptr(ld), 3,
                                      None, 0, C.byref(need), None) == 0
    # the diagonal-block inverses: 1 + 2 + 3 blocks of 2 x 64 x 64 doubles
    assert need.value >= 6 * 2 * 64 * 64 * 8
    assert lib.invaskit_getrs_batched(0, fake, binding._ptr(offs), binding._ptr(n), fake, fake,
                                      binding._ptr(boffs), binding._ptr(nr), binding._ptr(ld), 3,
                                      fake, need.value - 1, None, None) == binding.E_WORKSPACE
    assert lib.invaskit_getrf_batched(0, fake, binding._ptr(offs), binding._ptr(n), 3, fake, fake,
                                      None, 0, None, None) == binding.E_ARG

