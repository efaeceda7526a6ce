"""ctypes binding of libinvaskit.so (include/invaskit.h).

Argument marshalling only: every step of the factorization, solve and
product runs in the library's HIP kernels.  PyTorch supplies device memory
(the factor workspace, solve and product scratch, building-block workspaces:
uint8 tensors sized by the library's *_workspace_bytes queries) and the
current HIP stream.  Importing this module loads the library and fails
loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libinvaskit.so")

OK = 0
E_ARG, E_WORKSPACE, E_HIP, E_SINGULAR, E_NOT_CONVERGED, E_DEVICE = -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1


class InvaskitError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("depth", C.c_int32),
                ("points_dtype", C.c_int32), ("reserved0", C.c_int32),
                ("points", C.c_void_p), ("leaf_offsets", C.c_void_p),
                ("skel_offsets", C.c_void_p), ("skel_index", C.c_void_p),
                ("p_offsets", C.c_void_p), ("p_values", C.c_void_p), ("h", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("fp64_top_levels", C.c_int32),
                ("refine_tol", C.c_double), ("max_refine_iters", C.c_int32),
                ("tune", C.c_int32), ("leaf_lu_panel", C.c_int32),
                ("leaf_trsm_cols", C.c_int32), ("leaf_lu_waves", C.c_int32),
                ("refine", C.c_int32), ("gmres_restart", C.c_int32),
                ("max_gmres_iters", C.c_int32), ("lambda_group", C.c_int32),
                ("zlu_form", C.c_int32), ("zsolve_cols", C.c_int32),
                ("leaf_pivoting", C.c_int32)]


TUNE_AUTO, TUNE_OFF = 0, 1
REFINE = {"auto": 0, "ir": 1, "gmres": 2, "none": 3}
ZLU_FORM = {"auto": 0, "one_wave": 1, "block": 2}
LEAF_PIVOTING = {"auto": 0, "partial": 1}


class _TileConfig(C.Structure):
    _fields_ = [("leaf_lu_panel", C.c_int32), ("leaf_lu_waves", C.c_int32),
                ("leaf_trsm_cols", C.c_int32), ("tuned", C.c_int32),
                ("lu_ms", C.c_float * 4), ("trsm_ms", C.c_float * 2),
                ("leaf_trsm_cols_small", C.c_int32), ("trsm_small_ms", C.c_float * 2),
                ("zlu_one_wave_levels", C.c_int32), ("zsolve32_levels", C.c_int32),
                ("leaf_pivoting", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("final_rel_residual", C.c_double), ("unrefined_rel_residual", C.c_double),
                ("gmres_iterations", C.c_int32), ("method", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["method"] = {v: k for k, v in REFINE.items()}.get(d["method"], d["method"])
        return d


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_1602_01376_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sz, szp = C.c_size_t, C.POINTER(C.c_size_t)
    sig = {
        "invaskit_default_options": (C.c_int, [vp]),
        "invaskit_factor_workspace_bytes": (C.c_int, [vp, vp, i32, szp]),
        "invaskit_factor": (C.c_int, [vp, dbl, vp, vp, sz, vp, vp]),
        "invaskit_factor_sweep": (C.c_int, [vp, vp, i32, vp, vp, sz, vp, vp]),
        "invaskit_refactor": (C.c_int, [vp, dbl]),
        "invaskit_solve_workspace_bytes": (C.c_int, [vp, i64, szp, szp]),
        "invaskit_solve": (C.c_int, [vp, vp, i64, i64, vp, i64, vp, sz, vp]),
        "invaskit_matvec_workspace_bytes": (C.c_int, [vp, i64, szp]),
        "invaskit_matvec": (C.c_int, [vp, vp, i64, i64, vp, i64, vp, sz]),
        "invaskit_matvec_noalloc": (C.c_int, [vp, vp, i64, i64, vp, i64]),
        "invaskit_device_bytes": (C.c_int, [vp, szp]),
        "invaskit_phase_times": (C.c_int, [vp, vp, i32]),
        "invaskit_tile_config_get": (C.c_int, [vp, vp]),
        "invaskit_tuning_export": (C.c_int, [vp, C.c_size_t, vp]),
        "invaskit_tuning_import": (C.c_int, [C.c_char_p]),
        "invaskit_tuning_clear": (C.c_int, []),
        "invaskit_destroy": (C.c_int, [vp]),
        "invaskit_status_string": (C.c_char_p, [C.c_int]),
        "invaskit_last_error": (C.c_int, [vp, vp, C.c_size_t]),
        "invaskit_getrf_batched": (C.c_int, [i32, vp, vp, vp, i32, vp, vp, vp, sz, szp, vp]),
        "invaskit_getrs_batched": (C.c_int, [i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, sz,
                                             szp, vp]),
        "invaskit_kernel_blocks": (C.c_int, [i32, vp, i32, dbl, i32, vp, vp, vp, vp, vp, vp,
                                             vp, vp, dbl, i32, vp, sz, szp, vp]),
        "invaskit_gemm_batched": (C.c_int, [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                            vp, dbl, dbl, i32, vp, sz, szp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("invaskit_default_options", "invaskit_factor_workspace_bytes", "invaskit_factor",
            "invaskit_factor_sweep", "invaskit_refactor", "invaskit_solve_workspace_bytes",
            "invaskit_solve", "invaskit_matvec_workspace_bytes", "invaskit_matvec",
            "invaskit_matvec_noalloc",
            "invaskit_device_bytes", "invaskit_phase_times", "invaskit_tile_config_get",
            "invaskit_tuning_export", "invaskit_tuning_import", "invaskit_tuning_clear",
            "invaskit_destroy", "invaskit_status_string", "invaskit_last_error",
            "invaskit_getrf_batched", "invaskit_getrs_batched", "invaskit_kernel_blocks",
            "invaskit_gemm_batched")

# Above this many bytes of GMRES bases, a solve's scratch holds a shorter
# restart (the library uses the longest that fits; at least 2).
GMRES_SCRATCH_CAP = 4 << 30


def _device_buffer(nbytes: int) -> torch.Tensor:
    """Caller-owned device memory for the library: a uint8 tensor (the
    caching allocator aligns it to at least 256 bytes)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def library():
    return _lib


def last_error(handle=None) -> str:
    buf = C.create_string_buffer(1024)
    _lib.invaskit_last_error(handle, buf, 1024)
    return buf.value.decode(errors="replace")


def _check(status, handle=None):
    if status != OK:
        raise InvaskitError(status, last_error(handle) or
                            _lib.invaskit_status_string(status).decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _colmajor(t: torch.Tensor):
    """(N,) or (N, r) tensor -> (r, N) contiguous float64 on the GPU (its
    memory is the column-major N x r matrix)."""
    if t.dim() == 1:
        t = t[:, None]
    return t.to(device="cuda", dtype=torch.float64).t().contiguous()


class Factorization:
    """A factored lambda*I + K~ on the GPU (one library handle).

    `points` and `p_values` are borrowed by the library: this object keeps
    the device tensors alive for as long as the handle exists.  `tune`
    ("auto" or "off") and `leaf_lu_panel`, `leaf_lu_waves`, `leaf_trsm_cols`
    (0 = per `tune`) map to the tile options of invaskit_options;
    `tile_config()` reports what the factorization used.
    """

    def __init__(self, problem, lam: float, precision: str = "fp64",
                 fp64_top_levels: int = 4, refine_tol: float = 1e-10,
                 max_refine_iters: int = 30, points=None, p_values=None, tune: str = "auto",
                 leaf_lu_panel: int = 0, leaf_trsm_cols: int = 0, leaf_lu_waves: int = 0,
                 refine: str = "auto", gmres_restart: int = 20, max_gmres_iters: int = 300,
                 zlu_form: str = "auto", zsolve_cols: int = 0, leaf_pivoting: str = "auto"):
        pb, opt = self._prepare(problem, lam, precision, fp64_top_levels, refine_tol,
                                max_refine_iters, points, p_values, tune, leaf_lu_panel,
                                leaf_trsm_cols, leaf_lu_waves, refine, gmres_restart,
                                max_gmres_iters, zlu_form, zsolve_cols, leaf_pivoting)
        self._handle = C.c_void_p()
        need = C.c_size_t()
        _check(_lib.invaskit_factor_workspace_bytes(C.byref(pb), C.byref(opt), 0,
                                                    C.byref(need)))
        self._ws = _device_buffer(need.value)
        st = _lib.invaskit_factor(C.byref(pb), self.lam, C.byref(opt),
                                  C.c_void_p(self._ws.data_ptr()), self._ws.numel(), _stream(),
                                  C.byref(self._handle))
        if st != OK:
            msg = last_error(self._handle if self._handle.value else None)
            if self._handle.value:
                _lib.invaskit_destroy(self._handle)
                self._handle = C.c_void_p()
            raise InvaskitError(st, msg)

    def _prepare(self, problem, lam, precision, fp64_top_levels, refine_tol, max_refine_iters,
                 points, p_values, tune="auto", leaf_lu_panel=0, leaf_trsm_cols=0,
                 leaf_lu_waves=0, refine="auto", gmres_restart=20, max_gmres_iters=300,
                 zlu_form="auto", zsolve_cols=0, leaf_pivoting="auto"):
        """Marshal the problem and options (the arrays stay alive with self)."""
        self.n = problem.n
        self.lam = float(lam)
        self.precision = precision
        pdt = F32 if problem.X.dtype == np.float32 else F64
        if points is None:
            points = torch.from_numpy(np.ascontiguousarray(problem.X)).cuda()
        if p_values is None:
            p_values = torch.from_numpy(np.ascontiguousarray(problem.p_values, dtype=np.float64)).cuda()
        self._points = points
        self._p = p_values
        self._scratch = {}  # (kind, nrhs) -> caller-owned scratch of solves and products
        self._leaf = np.ascontiguousarray(problem.leaf_offsets, dtype=np.int64)
        self._so = np.ascontiguousarray(problem.skel_offsets, dtype=np.int64)
        self._si = np.ascontiguousarray(problem.skel_index, dtype=np.int32)
        self._po = np.ascontiguousarray(problem.p_offsets, dtype=np.int64)
        pb = _Problem(n=problem.n, d=problem.d, depth=problem.depth, points_dtype=pdt,
                      reserved0=0, points=points.data_ptr(), leaf_offsets=_ptr(self._leaf).value,
                      skel_offsets=_ptr(self._so).value, skel_index=_ptr(self._si).value,
                      p_offsets=_ptr(self._po).value, p_values=p_values.data_ptr(),
                      h=float(problem.h))
        opt = _Options()
        _lib.invaskit_default_options(C.byref(opt))
        opt.precision = PREC_MIXED if precision == "mixed" else PREC_FP64
        opt.fp64_top_levels = int(fp64_top_levels)
        opt.refine_tol = float(refine_tol)
        opt.max_refine_iters = int(max_refine_iters)
        if tune not in ("auto", "off"):
            raise ValueError("tune must be 'auto' or 'off'")
        opt.tune = TUNE_OFF if tune == "off" else TUNE_AUTO
        opt.leaf_lu_panel = int(leaf_lu_panel)
        opt.leaf_trsm_cols = int(leaf_trsm_cols)
        opt.leaf_lu_waves = int(leaf_lu_waves)
        if refine not in REFINE:
            raise ValueError(f"refine must be one of {sorted(REFINE)}")
        opt.refine = REFINE[refine]
        opt.gmres_restart = int(gmres_restart)
        opt.max_gmres_iters = int(max_gmres_iters)
        if zlu_form not in ZLU_FORM:
            raise ValueError(f"zlu_form must be one of {sorted(ZLU_FORM)}")
        opt.zlu_form = ZLU_FORM[zlu_form]
        opt.zsolve_cols = int(zsolve_cols)
        if leaf_pivoting not in LEAF_PIVOTING:
            raise ValueError(f"leaf_pivoting must be one of {sorted(LEAF_PIVOTING)}")
        opt.leaf_pivoting = LEAF_PIVOTING[leaf_pivoting]
        return pb, opt

    @property
    def handle(self):
        return self._handle

    def refactor(self, lam: float):
        self.lam = float(lam)
        _check(_lib.invaskit_refactor(self._handle, self.lam), self._handle)

    def scratch(self, kind: str, r: int) -> torch.Tensor:
        """The scratch this object passes to invaskit_solve ("solve") or
        invaskit_matvec ("matvec") for r columns: allocated on first use and
        kept, so the library reuses the descriptor tables it left there."""
        key = (kind, int(r))
        if key not in self._scratch:
            full, low = C.c_size_t(), C.c_size_t()
            if kind == "solve":
                _check(_lib.invaskit_solve_workspace_bytes(self._handle, r, C.byref(full),
                                                           C.byref(low)), self._handle)
                nbytes = full.value if full.value - low.value <= GMRES_SCRATCH_CAP \
                    else low.value + GMRES_SCRATCH_CAP
            else:
                _check(_lib.invaskit_matvec_workspace_bytes(self._handle, r, C.byref(full)),
                       self._handle)
                nbytes = full.value
            self._scratch[key] = _device_buffer(nbytes)
        return self._scratch[key]

    def solve(self, b: torch.Tensor, return_info: bool = False, check: bool = True):
        """x = (lambda I + K~)^-1 b for b of shape (N,) or (N, r) (tree order)."""
        vec = b.dim() == 1
        bc = _colmajor(b)
        r = bc.shape[0]
        xc = torch.empty_like(bc)
        info = SolveInfo()
        sc = self.scratch("solve", r)
        st = _lib.invaskit_solve(self._handle, C.c_void_p(bc.data_ptr()), r, self.n,
                                 C.c_void_p(xc.data_ptr()), self.n, C.c_void_p(sc.data_ptr()),
                                 sc.numel(), C.byref(info) if return_info else None)
        if check:
            _check(st, self._handle)
        x = xc.t()
        if vec:
            x = x[:, 0]
        if return_info:
            return x, info.as_dict(), st
        return x

    def matvec(self, x: torch.Tensor):
        """y = (lambda I + K~) x in FP64."""
        vec = x.dim() == 1
        xc = _colmajor(x)
        r = xc.shape[0]
        yc = torch.empty_like(xc)
        sc = self.scratch("matvec", r)
        _check(_lib.invaskit_matvec(self._handle, C.c_void_p(xc.data_ptr()), r, self.n,
                                    C.c_void_p(yc.data_ptr()), self.n, C.c_void_p(sc.data_ptr()),
                                    sc.numel()), self._handle)
        y = yc.t()
        return y[:, 0] if vec else y

    def phase_times(self):
        out = (C.c_double * 12)()
        _check(_lib.invaskit_phase_times(self._handle, out, 12), self._handle)
        keys = ["leaf_blocks", "leaf_lu", "leaf_diag_inverses", "skeleton_blocks", "leaf_solves",
                "leaf_projections", "skeleton_sweep", "handle_planning", "reduced_systems",
                "total", "leaf_lu_large", "leaf_solves_large"]
        return dict(zip(keys, list(out)))

    def tile_config(self):
        """Tile shapes of the last factor (invaskit_tile_config_get)."""
        t = _TileConfig()
        _check(_lib.invaskit_tile_config_get(self._handle, C.byref(t)), self._handle)
        return {"leaf_lu_panel": t.leaf_lu_panel, "leaf_lu_waves": t.leaf_lu_waves,
                "leaf_trsm_cols": t.leaf_trsm_cols, "tuned": t.tuned, "lu_ms": list(t.lu_ms),
                "trsm_ms": list(t.trsm_ms), "leaf_trsm_cols_small": t.leaf_trsm_cols_small,
                "trsm_small_ms": list(t.trsm_small_ms),
                "zlu_one_wave_levels": t.zlu_one_wave_levels,
                "zsolve32_levels": t.zsolve32_levels, "leaf_pivoting": t.leaf_pivoting}

    def device_bytes(self):
        """Bytes of the factor workspace this handle's buffers span."""
        v = C.c_size_t()
        _check(_lib.invaskit_device_bytes(self._handle, C.byref(v)), self._handle)
        return v.value

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.invaskit_destroy(self._handle)
            self._handle = C.c_void_p()
        # the workspace and scratch go after the handle that used them
        self._scratch = {}
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------ batched building blocks
def _block_workspace(fn, args):
    """Query a building block's workspace size (workspace = NULL) and
    allocate it."""
    need = C.c_size_t()
    _check(fn(*args, None, 0, C.byref(need), _stream()))
    return _device_buffer(need.value)


def getrf_batched(mats, dtype=torch.float64):
    """LU with partial pivoting of a list of square matrices (numpy or torch,
    any size 1..1024) in one launch.  Returns (packed row-major factors,
    offsets, sizes, perm, info)."""
    ns = [int(m.shape[0]) for m in mats]
    offs = np.zeros(len(mats), dtype=np.int64)
    off = 0
    parts = []
    for i, m in enumerate(mats):
        offs[i] = off
        off += ns[i] * ns[i]
        parts.append(torch.as_tensor(np.asarray(m)).to(dtype).contiguous().reshape(-1))  # row-major
    buf = torch.cat(parts).cuda()
    perm = torch.empty(sum(ns), dtype=torch.int32, device="cuda")
    info = torch.empty(len(mats), dtype=torch.int32, device="cuda")
    n_arr = np.asarray(ns, dtype=np.int32)
    dt = F64 if dtype == torch.float64 else F32
    args = (dt, C.c_void_p(buf.data_ptr()), _ptr(offs), _ptr(n_arr), len(mats),
            C.c_void_p(perm.data_ptr()), C.c_void_p(info.data_ptr()))
    ws = _block_workspace(_lib.invaskit_getrf_batched, args)
    _check(_lib.invaskit_getrf_batched(*args, C.c_void_p(ws.data_ptr()), ws.numel(), None,
                                       _stream()))
    return buf, offs, n_arr, perm, info


def getrs_batched(buf, offs, n_arr, perm, rhs_list, dtype=torch.float64):
    """Solve with factors from getrf_batched; rhs_list[i] is (n_i, r_i)."""
    boffs = np.zeros(len(rhs_list), dtype=np.int64)
    nr = np.zeros(len(rhs_list), dtype=np.int32)
    ld = np.zeros(len(rhs_list), dtype=np.int64)
    parts = []
    off = 0
    for i, b in enumerate(rhs_list):
        bt = torch.as_tensor(np.asarray(b)).to(dtype)
        if bt.dim() == 1:
            bt = bt[:, None]
        boffs[i] = off
        nr[i] = bt.shape[1]
        ld[i] = bt.shape[0]
        off += bt.numel()
        parts.append(bt.t().contiguous().reshape(-1))
    bb = torch.cat(parts).cuda()
    dt = F64 if dtype == torch.float64 else F32
    args = (dt, C.c_void_p(buf.data_ptr()), _ptr(offs), _ptr(n_arr), C.c_void_p(perm.data_ptr()),
            C.c_void_p(bb.data_ptr()), _ptr(boffs), _ptr(nr), _ptr(ld), len(rhs_list))
    ws = _block_workspace(_lib.invaskit_getrs_batched, args)
    _check(_lib.invaskit_getrs_batched(*args, C.c_void_p(ws.data_ptr()), ws.numel(), None,
                                       _stream()))
    out = []
    for i in range(len(rhs_list)):
        seg = bb[boffs[i]:boffs[i] + nr[i] * ld[i]].reshape(int(nr[i]), int(ld[i])).t()
        out.append(seg)
    return out


def kernel_blocks(points: torch.Tensor, h: float, blocks, out_dtype=torch.float64, shift=0.0):
    """Evaluate Gaussian kernel blocks; blocks = [(row0, rows, col_ids, diag)]."""
    d = int(points.shape[1])
    pdt = F32 if points.dtype == torch.float32 else F64
    odt = F64 if out_dtype == torch.float64 else F32
    cnt = len(blocks)
    out_off = np.zeros(cnt, np.int64)
    row0 = np.zeros(cnt, np.int64)
    rows = np.zeros(cnt, np.int32)
    ncols = np.zeros(cnt, np.int32)
    coff = np.zeros(cnt, np.int64)
    diag = np.zeros(cnt, np.int32)
    cols = []
    o = c = 0
    for i, (r0, nr, cid, dg) in enumerate(blocks):
        out_off[i], row0[i], rows[i], ncols[i], coff[i], diag[i] = o, r0, nr, len(cid), c, int(dg)
        o += nr * len(cid)
        c += len(cid)
        cols.append(np.asarray(cid, dtype=np.int32))
    cols_t = torch.from_numpy(np.concatenate(cols) if cols else np.zeros(1, np.int32)).cuda()
    out = torch.empty(max(o, 1), dtype=out_dtype, device="cuda")
    args = (pdt, C.c_void_p(points.data_ptr()), d, float(h), odt, C.c_void_p(out.data_ptr()),
            _ptr(out_off), _ptr(row0), _ptr(rows), C.c_void_p(cols_t.data_ptr()), _ptr(coff),
            _ptr(ncols), _ptr(diag), float(shift), cnt)
    ws = _block_workspace(_lib.invaskit_kernel_blocks, args)
    _check(_lib.invaskit_kernel_blocks(*args, C.c_void_p(ws.data_ptr()), ws.numel(), None,
                                       _stream()))
    res = []
    for i in range(cnt):
        res.append(out[out_off[i]:out_off[i] + rows[i] * ncols[i]]
                   .reshape(int(ncols[i]), int(rows[i])).t())
    return res


def gemm_batched(problems, dtype=torch.float64, alpha=1.0, beta=0.0):
    """problems = [(A, B, C0, a_rowmajor)] with numpy A (m x k), B (k x n),
    C0 (m x n or None).  Returns the list of C = beta*C0 + alpha*A B."""
    cnt = len(problems)
    a_off, b_off, c_off = (np.zeros(cnt, np.int64) for _ in range(3))
    m, n, k, arm = (np.zeros(cnt, np.int32) for _ in range(4))
    lda, ldb, ldc = (np.zeros(cnt, np.int64) for _ in range(3))
    pa, pb_, pc = [], [], []
    oa = ob = oc = 0
    for i, (A, B, C0, rm) in enumerate(problems):
        A = np.asarray(A)
        B = np.asarray(B)
        m[i], k[i] = A.shape
        n[i] = B.shape[1]
        arm[i] = int(rm)
        a_off[i], b_off[i], c_off[i] = oa, ob, oc
        if rm:
            pa.append(torch.as_tensor(A).to(dtype).contiguous().reshape(-1))
            lda[i] = max(k[i], 1)
        else:
            pa.append(torch.as_tensor(A).to(dtype).t().contiguous().reshape(-1))
            lda[i] = max(m[i], 1)
        pb_.append(torch.as_tensor(B).to(dtype).t().contiguous().reshape(-1))
        ldb[i] = max(k[i], 1)
        C0 = np.zeros((m[i], n[i])) if C0 is None else np.asarray(C0)
        pc.append(torch.as_tensor(C0).to(dtype).t().contiguous().reshape(-1))
        ldc[i] = max(m[i], 1)
        oa += A.size
        ob += B.size
        oc += m[i] * n[i]
    ta = torch.cat(pa + [torch.zeros(1, dtype=dtype)]).cuda()
    tb = torch.cat(pb_ + [torch.zeros(1, dtype=dtype)]).cuda()
    tc = torch.cat(pc + [torch.zeros(1, dtype=dtype)]).cuda()
    dt = F64 if dtype == torch.float64 else F32
    args = (dt, C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), C.c_void_p(tc.data_ptr()),
            _ptr(a_off), _ptr(b_off), _ptr(c_off), _ptr(m), _ptr(n), _ptr(k), _ptr(lda), _ptr(arm),
            _ptr(ldb), _ptr(ldc), float(alpha), float(beta), cnt)
    ws = _block_workspace(_lib.invaskit_gemm_batched, args)
    _check(_lib.invaskit_gemm_batched(*args, C.c_void_p(ws.data_ptr()), ws.numel(), None,
                                      _stream()))
    out = []
    for i in range(cnt):
        out.append(tc[c_off[i]:c_off[i] + m[i] * n[i]].reshape(int(n[i]), int(m[i])).t())
    return out


def factor_sweep(problem, lams, precision: str = "fp64", fp64_top_levels: int = 4,
                 refine_tol: float = 1e-10, max_refine_iters: int = 30, points=None,
                 p_values=None, tune: str = "auto", leaf_lu_panel: int = 0,
                 leaf_trsm_cols: int = 0, leaf_lu_waves: int = 0, refine: str = "auto",
                 gmres_restart: int = 20, max_gmres_iters: int = 300, lambda_group: int = 0,
                 zlu_form: str = "auto", zsolve_cols: int = 0, leaf_pivoting: str = "auto"):
    """One Factorization per lambda in `lams` (invaskit_factor_sweep): the
    kernel blocks are evaluated once into the sweep's workspace and shared
    by the handles; the lambdas are factored in batches of `lambda_group`
    (0: all together), each batch in one set of launches."""
    lams = [float(v) for v in lams]
    objs = [Factorization.__new__(Factorization) for _ in lams]
    pb, opt = objs[0]._prepare(problem, lams[0], precision, fp64_top_levels, refine_tol,
                               max_refine_iters, points, p_values, tune, leaf_lu_panel,
                               leaf_trsm_cols, leaf_lu_waves, refine, gmres_restart,
                               max_gmres_iters, zlu_form, zsolve_cols, leaf_pivoting)
    opt.lambda_group = int(lambda_group)
    need = C.c_size_t()
    _check(_lib.invaskit_factor_workspace_bytes(C.byref(pb), C.byref(opt), len(lams),
                                                C.byref(need)))
    ws = _device_buffer(need.value)
    for o, lam in zip(objs[1:], lams[1:]):
        o.n, o.lam, o.precision = objs[0].n, lam, precision
        o._points, o._p = objs[0]._points, objs[0]._p
        o._keep = objs[0]
        o._scratch = {}
    for o in objs:
        o._ws = ws  # shared: freed with the last of them
    arr = (C.c_double * len(lams))(*lams)
    handles = (C.c_void_p * len(lams))()
    st = _lib.invaskit_factor_sweep(C.byref(pb), arr, len(lams), C.byref(opt),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream(), handles)
    for o, hnd in zip(objs, handles):
        o._handle = C.c_void_p(hnd)
    if st != OK:
        msg = last_error(next((C.c_void_p(hd) for hd in handles if hd), None))
        for o in objs:
            o.close()
        raise InvaskitError(st, msg)
    return objs


# ------------------------------------------------------------- tuning table
def tuning_table() -> dict:
    """The process-wide tile tuning table as {shape class: choice}."""
    need = C.c_size_t()
    _check(_lib.invaskit_tuning_export(None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(_lib.invaskit_tuning_export(buf, need.value, C.byref(need)))
    out = {}
    for line in buf.value.decode().splitlines():
        k, v = line.split()
        out[k] = int(v)
    return out


def tuning_load(entries: dict):
    """Add {shape class: choice} entries to the tuning table."""
    text = "".join(f"{k} {int(v)}\n" for k, v in entries.items())
    _check(_lib.invaskit_tuning_import(text.encode()))


def tuning_clear():
    _check(_lib.invaskit_tuning_clear())


def _arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def save_tuning(path: str):
    """Write the tuning table to a JSON file, keyed by the GPU architecture
    (other architectures' entries in the file are kept)."""
    import json
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[_arch()] = tuning_table()
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_tuning(path: str) -> int:
    """Load this architecture's entries of a save_tuning file; returns how
    many were loaded."""
    import json
    with open(path) as f:
        entries = json.load(f).get(_arch(), {})
    tuning_load(entries)
    return len(entries)
