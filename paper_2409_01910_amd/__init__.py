"""Python binding of libbz, the MI355X (gfx950) steady-state Boltzmann hot path.

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are torch CUDA (HIP) tensors on the context's device;
their raw pointers and the current HIP stream are handed to the C ABI
declared in ``include/bz.h``.  If ``libbz.so`` is missing, importing the
collision entry points raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbz.so")

BZ_FP64, BZ_FP32, BZ_FP32_DIFF = 0, 1, 2
BZ_ENUMERIC = 5
BZ_METHOD_SIGMA, BZ_METHOD_CARLEMAN = 0, 1
BZ_Q_CORRECTED = 1
BZ_Q_MASS = 2
BZ_Q_CONSERVE = 4
BZ_BC_WALL, BZ_BC_INFLOW = 0, 1
BZ_SOLVE_PFP, BZ_SOLVE_FP, BZ_SOLVE_SI = 0, 1, 2
BZ_COLL_BINARY, BZ_COLL_BGK, BZ_COLL_BINARY_CONSERVE = 0, 1, 2
_COLLISIONS = {"binary": BZ_COLL_BINARY, "bgk": BZ_COLL_BGK, "binary_conserve": BZ_COLL_BINARY_CONSERVE}
_LIMITERS = {"none": 0, "minmod": 1}

# every symbol include/bz.h declares
EXPORTED = [
    "bz_create", "bz_destroy", "bz_status_str", "bz_last_error", "bz_workspace_bytes",
    "bz_eval_Q", "bz_eval_Q_noalloc", "bz_maxwellian", "bz_cell_solve", "bz_cell_fixed_point",
    "bz_slab_create", "bz_slab_destroy", "bz_sgs_sweep", "bz_outer_residual", "bz_multigrid_vcycle",
    "bz_profile_enable", "bz_profile_get",
    "bz_mlp_create", "bz_mlp_destroy", "bz_mlp_num_params", "bz_mlp_get_params", "bz_mlp_set_params",
    "bz_mlp_set_output_scale", "bz_mlp_forward", "bz_mlp_grad", "bz_mlp_train_step", "bz_mlp_features",
    "bz_cell_fixed_point_learned",
    "bz_graph_capture_sweeps", "bz_graph_capture_vcycles", "bz_graph_launch", "bz_graph_destroy",
    "bz_cavity_create", "bz_cavity_destroy", "bz_cavity_sweep", "bz_cavity_residual", "bz_cavity_vcycle",
    "bz_slab_inflow", "bz_ws_attach", "bz_set_plan", "bz_get_plan", "bz_tune",
    "bz_cavity_inflow", "bz_cavity_ws_attach", "bz_eval_Q_strided", "bz_cell_fixed_point_ex", "bz_set_strict",
    "bz_cell_check",
]


class bz_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("L", ctypes.c_double), ("gamma", ctypes.c_double),
                ("n_theta", ctypes.c_int), ("n_phi", ctypes.c_int), ("n_rho", ctypes.c_int),
                ("R", ctypes.c_double), ("precision", ctypes.c_int), ("device", ctypes.c_int),
                ("v1_shift", ctypes.c_double), ("method", ctypes.c_int), ("d", ctypes.c_int)]


class bz_solve_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("fixed_iters", ctypes.c_int), ("fallback", ctypes.c_int)]


class bz_cell_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("fallback", ctypes.c_int32), ("newton_fail", ctypes.c_int32),
                ("status", ctypes.c_int32), ("residual", ctypes.c_double), ("learned", ctypes.c_int32),
                ("relaxed", ctypes.c_int32)]


class bz_slab_instance(ctypes.Structure):
    _fields_ = [("xL", ctypes.c_double), ("xR", ctypes.c_double), ("nx", ctypes.c_int), ("eps", ctypes.c_double),
                ("T_L", ctypes.c_double), ("T_R", ctypes.c_double), ("U_L", ctypes.c_double * 3),
                ("U_R", ctypes.c_double * 3), ("mass", ctypes.c_double), ("bc_L", ctypes.c_int),
                ("bc_R", ctypes.c_int), ("rho_L", ctypes.c_double), ("rho_R", ctypes.c_double)]


class bz_slab_desc(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int), ("instances", ctypes.POINTER(bz_slab_instance)),
                ("collision", ctypes.c_int), ("bgk_nu", ctypes.c_double), ("inner", bz_solve_opts),
                ("f", ctypes.c_void_p), ("order", ctypes.c_int), ("limiter", ctypes.c_int)]


class bz_wall(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("U", ctypes.c_double * 2)]


class bz_cavity_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("eps", ctypes.c_double), ("walls", bz_wall * 4),
                ("mass", ctypes.c_double), ("collision", ctypes.c_int), ("bgk_nu", ctypes.c_double),
                ("inner", bz_solve_opts), ("f", ctypes.c_void_p), ("order", ctypes.c_int),
                ("uniform_y", ctypes.c_int), ("limiter", ctypes.c_int)]


class bz_sweep_stats(ctypes.Structure):
    _fields_ = [("n_iters", ctypes.c_int), ("inner_iters", ctypes.c_int64), ("visits", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("learned", ctypes.c_int64)]


class bz_mg_opts(ctypes.Structure):
    _fields_ = [("coarsest", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("coarse_iters", ctypes.c_int), ("tol", ctypes.c_double), ("fixed_cycle", ctypes.c_int)]


class bz_plan(ctypes.Structure):
    _fields_ = [("pair_waves", ctypes.c_int), ("chunk_cells", ctypes.c_int), ("acc_nodes", ctypes.c_int)]


BZ_TUNE_MAX = 16


class bz_tune_report(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("plan", bz_plan * BZ_TUNE_MAX), ("ms", ctypes.c_double * BZ_TUNE_MAX),
                ("best", ctypes.c_int)]


class bz_profile_info(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("flops", ctypes.c_double)]


CELL_STATS_DTYPE_FIELDS = [("iterations", "<i4"), ("fallback", "<i4"), ("newton_fail", "<i4"), ("status", "<i4"),
                           ("residual", "<f8"), ("learned", "<i4"), ("relaxed", "<i4")]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbz.so and declare argument types.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libbz.so not built at {path}: run __graft_entry__.build()")
    # torch first (when installed), so that the library binds to the HIP
    # runtime torch loads and the process holds one runtime, whichever of the
    # two the caller imports first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I64, D, U32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.bz_create.argtypes = [ctypes.POINTER(bz_params), ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_destroy.argtypes = [P]
    lib.bz_destroy.restype = None
    lib.bz_status_str.argtypes = [ctypes.c_int]
    lib.bz_status_str.restype = ctypes.c_char_p
    lib.bz_last_error.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
    lib.bz_workspace_bytes.argtypes = [P]
    lib.bz_workspace_bytes.restype = ctypes.c_size_t
    lib.bz_eval_Q.argtypes = [P, P, P, I64, U32, P, P]
    lib.bz_eval_Q_noalloc.argtypes = [P, P, P, I64, U32, P, P]
    lib.bz_eval_Q_strided.argtypes = [P, P, I64, P, I64, I64, U32, P, P]
    lib.bz_cell_fixed_point_ex.argtypes = [P, P, P, P, P, D, P, P, P, I64, ctypes.POINTER(bz_solve_opts), P, P]
    lib.bz_set_strict.argtypes = [P, ctypes.c_int]
    lib.bz_cell_check.argtypes = [P, P, I64, ctypes.POINTER(I64), P]
    lib.bz_maxwellian.argtypes = [P, P, P, P, P, I64, P]
    lib.bz_cell_solve.argtypes = [P, P, P, P, D, P, P, I64, ctypes.POINTER(bz_solve_opts), P, P]
    lib.bz_cell_fixed_point.argtypes = [P, P, P, P, D, P, I64, ctypes.POINTER(bz_solve_opts), P, P]
    lib.bz_slab_create.argtypes = [P, ctypes.POINTER(bz_slab_desc), ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_slab_destroy.argtypes = [P]
    lib.bz_slab_destroy.restype = None
    lib.bz_sgs_sweep.argtypes = [P, P, ctypes.c_int, P, ctypes.POINTER(bz_sweep_stats), P]
    lib.bz_cavity_create.argtypes = [P, ctypes.POINTER(bz_cavity_desc), ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_cavity_destroy.argtypes = [P]
    lib.bz_cavity_destroy.restype = None
    lib.bz_cavity_sweep.argtypes = [P, P, ctypes.c_int, P, ctypes.POINTER(bz_sweep_stats), P]
    lib.bz_cavity_residual.argtypes = [P, P, P, P]
    lib.bz_cavity_vcycle.argtypes = [P, P, ctypes.POINTER(bz_mg_opts), ctypes.c_int, P,
                                     ctypes.POINTER(bz_sweep_stats), P]
    lib.bz_outer_residual.argtypes = [P, P, P, P]
    lib.bz_slab_inflow.argtypes = [P, P, P, P]
    lib.bz_ws_attach.argtypes = [P, P]
    lib.bz_cavity_inflow.argtypes = [P, P, P, P]
    lib.bz_cavity_ws_attach.argtypes = [P, P]
    lib.bz_multigrid_vcycle.argtypes = [P, P, ctypes.POINTER(bz_mg_opts), ctypes.c_int, P,
                                        ctypes.POINTER(bz_sweep_stats), P]
    lib.bz_mlp_create.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_mlp_destroy.argtypes = [P]
    lib.bz_mlp_destroy.restype = None
    lib.bz_mlp_num_params.argtypes = [P]
    lib.bz_mlp_num_params.restype = ctypes.c_int64
    lib.bz_mlp_get_params.argtypes = [P, P, I64]
    lib.bz_mlp_set_params.argtypes = [P, P, I64]
    lib.bz_mlp_set_output_scale.argtypes = [P, D]
    lib.bz_mlp_forward.argtypes = [P, P, P, I64, ctypes.c_int, P]
    lib.bz_mlp_grad.argtypes = [P, P, P, I64, P, ctypes.POINTER(ctypes.c_double), P]
    lib.bz_mlp_train_step.argtypes = [P, P, P, I64, D, ctypes.POINTER(ctypes.c_double), P]
    lib.bz_mlp_features.argtypes = [P, P, P, P, D, P, I64, P]
    lib.bz_cell_fixed_point_learned.argtypes = [P, P, P, P, P, D, P, I64, ctypes.POINTER(bz_solve_opts), P, P]
    lib.bz_set_plan.argtypes = [P, ctypes.POINTER(bz_plan)]
    lib.bz_get_plan.argtypes = [P, ctypes.POINTER(bz_plan)]
    lib.bz_tune.argtypes = [P, P, I64, U32, ctypes.c_int, ctypes.POINTER(bz_tune_report), P]
    lib.bz_profile_enable.argtypes = [P, ctypes.c_int]
    lib.bz_profile_get.argtypes = [P, ctypes.POINTER(bz_profile_info)]
    lib.bz_graph_capture_sweeps.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_graph_capture_vcycles.argtypes = [P, P, ctypes.POINTER(bz_mg_opts), ctypes.c_int, ctypes.c_int, P,
                                             ctypes.POINTER(ctypes.c_void_p)]
    lib.bz_graph_launch.argtypes = [P, P, ctypes.POINTER(bz_sweep_stats), P]
    lib.bz_graph_destroy.argtypes = [P]
    lib.bz_graph_destroy.restype = None
    for name in EXPORTED:
        if name not in ("bz_destroy", "bz_slab_destroy", "bz_status_str", "bz_workspace_bytes", "bz_mlp_destroy",
                        "bz_graph_destroy", "bz_cavity_destroy",
                        "bz_mlp_num_params"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class BZError(RuntimeError):
    pass


class BZNumericError(BZError):
    """BZ_ENUMERIC: strict mode found a non-finite result (the call's outputs are filled)."""


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _arg(t, name, numel, dtype="float64", device=None, optional=False):
    """Check a tensor argument before its pointer reaches the library: a
    contiguous device tensor of the given dtype with exactly ``numel`` elements
    (on ``device`` when given).  Raises BZError otherwise; None passes only
    when ``optional``."""
    import torch

    if t is None:
        if optional:
            return None
        raise BZError(f"{name} is required")
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor) or t.dtype != want or not t.is_cuda or not t.is_contiguous():
        raise BZError(f"{name} must be a contiguous {dtype} device tensor")
    if device is not None and t.device != device:
        raise BZError(f"{name} is on {t.device}, expected {device}")
    if t.numel() != numel:
        raise BZError(f"{name} has {t.numel()} elements, expected {numel}")
    return t


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Params:
    N: int = 32
    L: float = 8.0
    gamma: float = 0.0
    n_theta: int = 8
    n_phi: int = 16
    n_rho: int = 16
    R: float = 0.0
    precision: int = BZ_FP64
    device: int = 0
    v1_shift: float = 0.0  # physical v_1 of the grid origin (transport uses node + v1_shift)
    method: int = 0  # BZ_METHOD_SIGMA, or BZ_METHOD_CARLEMAN (hard spheres, gamma = 1)
    d: int = 3  # velocity dimension (3, or 2: N x N grid, n_phi circle directions)


class Context:
    """Owns a bz_ctx.  Tensors passed to it must be float64, contiguous, on cuda:device."""

    def __init__(self, params: Params | None = None, **kw):
        self.lib = load_library()
        self.params = params or Params(**kw)
        p = bz_params(self.params.N, self.params.L, self.params.gamma, self.params.n_theta, self.params.n_phi,
                      self.params.n_rho, self.params.R, self.params.precision, self.params.device,
                      self.params.v1_shift, self.params.method, self.params.d)
        h = ctypes.c_void_p()
        st = self.lib.bz_create(ctypes.byref(p), ctypes.byref(h))
        if st != 0:
            raise BZError(f"bz_create: {self.lib.bz_status_str(st).decode()}")
        self.h = h
        self.d = self.params.d
        self.K = self.params.N ** self.d

    def close(self):
        if getattr(self, "h", None):
            self.lib.bz_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            buf = ctypes.create_string_buffer(512)
            self.lib.bz_last_error(self.h, buf, 512)
            cls = BZNumericError if st == BZ_ENUMERIC else BZError
            raise cls(f"{what}: {self.lib.bz_status_str(st).decode()}: {buf.value.decode()}")

    def _field(self, t, name):
        import torch

        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise BZError(f"{name} must be a contiguous float64 device tensor")
        if t.device.index != self.params.device:
            raise BZError(f"{name} is on {t.device}, the context on cuda:{self.params.device}")
        if t.numel() % self.K:
            raise BZError(f"{name}: size not a multiple of K = {self.K}")
        return t.numel() // self.K

    def eval_Q(self, f, corrected: bool = True, out=None, theta=None, conserve: str | None = None):
        """conserve: None, "mass" (BZ_Q_MASS) or "all" (BZ_Q_CONSERVE)."""
        import torch

        B = self._field(f, "f")
        Q = torch.empty_like(f) if out is None else _arg(out, "out", f.numel(), device=f.device)
        _arg(theta, "theta", B * (self.d + 2), device=f.device, optional=True)
        flags = (BZ_Q_CORRECTED if corrected else 0) | {None: 0, "mass": BZ_Q_MASS, "all": BZ_Q_CONSERVE}[conserve]
        st = self.lib.bz_eval_Q(self.h, _ptr(f), _ptr(Q), B, flags, _ptr(theta), _stream())
        self._check(st, "bz_eval_Q")
        return Q

    def eval_Q_strided(self, f, out, corrected: bool = True, theta=None, conserve: str | None = None):
        """bz_eval_Q_strided: f and out are float64 device views [batch, K] with
        unit stride along K and row strides >= K (e.g. every other row of a
        larger array)."""
        import torch

        for t, n in ((f, "f"), (out, "out")):
            if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2
                    or t.shape[1] != self.K or t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < self.K)
                    or t.device != f.device):
                raise BZError(f"{n} must be a float64 device view [batch, K] with unit inner stride")
        B = f.shape[0]
        if out.shape[0] != B:
            raise BZError("out must have the batch of f")
        _arg(theta, "theta", B * (self.d + 2), device=f.device, optional=True)
        flags = (BZ_Q_CORRECTED if corrected else 0) | {None: 0, "mass": BZ_Q_MASS, "all": BZ_Q_CONSERVE}[conserve]
        ldf = f.stride(0) if B > 1 else self.K
        ldq = out.stride(0) if B > 1 else self.K
        st = self.lib.bz_eval_Q_strided(self.h, _ptr(f), ldf, _ptr(out), ldq, B, flags, _ptr(theta), _stream())
        self._check(st, "bz_eval_Q_strided")
        return out

    def set_strict(self, on: bool = True):
        """bz_set_strict: calls that return residuals raise BZNumericError on a non-finite one."""
        self._check(self.lib.bz_set_strict(self.h, 1 if on else 0), "bz_set_strict")

    def cell_check(self, stats):
        """bz_cell_check: cells of a cell call's statistics that ended non-finite
        (synchronises; raises BZNumericError in strict mode when there is one)."""
        n = ctypes.c_int64(0)
        B = stats.numel() * stats.element_size() // ctypes.sizeof(bz_cell_stats)
        self._check(self.lib.bz_cell_check(self.h, _ptr(stats), B, ctypes.byref(n), _stream()), "bz_cell_check")
        return n.value

    def eval_Q_noalloc(self, f, out, corrected: bool = True, theta=None, conserve: str | None = None):
        """bz_eval_Q_noalloc: the collision term into the caller's ``out`` with no
        device allocation, neither by the library nor here."""
        B = self._field(f, "f")
        _arg(out, "out", f.numel(), device=f.device)
        _arg(theta, "theta", B * (self.d + 2), device=f.device, optional=True)
        flags = (BZ_Q_CORRECTED if corrected else 0) | {None: 0, "mass": BZ_Q_MASS, "all": BZ_Q_CONSERVE}[conserve]
        st = self.lib.bz_eval_Q_noalloc(self.h, _ptr(f), _ptr(out), B, flags, _ptr(theta), _stream())
        self._check(st, "bz_eval_Q_noalloc")
        return out

    def maxwellian(self, f, want_M: bool = True):
        import torch

        B = self._field(f, "f")
        theta = torch.empty((B, self.d + 2), dtype=torch.float64, device=f.device)
        M = torch.empty_like(f) if want_M else None
        it = torch.empty(B, dtype=torch.int32, device=f.device)
        st = self.lib.bz_maxwellian(self.h, _ptr(f), _ptr(theta), _ptr(M), _ptr(it), B, _stream())
        self._check(st, "bz_maxwellian")
        return theta, M, it

    @staticmethod
    def _opts(mode="pfp", tol=1e-8, max_iter=100, fixed_iters=0, fallback="fp"):
        """fallback: "fp" (the plain iteration) or "relax" (the relaxed step 1)."""
        modes = {"pfp": BZ_SOLVE_PFP, "fp": BZ_SOLVE_FP, "si": BZ_SOLVE_SI}
        if mode not in modes or fallback not in ("fp", "relax"):
            raise ValueError(f"mode must be one of {sorted(modes)} and fallback 'fp' or 'relax'")
        return bz_solve_opts(modes[mode], tol, max_iter, fixed_iters, {"fp": 0, "relax": 1}[fallback])

    @staticmethod
    def _stats_tensor(B, device):
        import torch

        return torch.zeros((B, 4), dtype=torch.float64, device=device)  # 32 bytes per cell

    @staticmethod
    def decode_stats(t):
        import numpy as np

        raw = t.detach().cpu().numpy().tobytes()
        return np.frombuffer(raw, dtype=np.dtype(CELL_STATS_DTYPE_FIELDS))

    def cell_solve(self, r, nu, eps, dx, g0, mode="pfp", tol=1e-8, max_iter=100, fixed_iters=0, out=None,
                   fallback="fp"):
        import torch

        B = self._field(r, "r")
        for t, n, k in ((nu, "nu", B), (eps, "eps", B), (g0, "g0", B * self.K)):
            _arg(t, n, k, device=r.device)
        g = torch.empty_like(r) if out is None else _arg(out, "out", r.numel(), device=r.device)
        stats = self._stats_tensor(B, r.device)
        o = self._opts(mode, tol, max_iter, fixed_iters, fallback)
        st = self.lib.bz_cell_solve(self.h, _ptr(r), _ptr(nu), _ptr(eps), float(dx), _ptr(g0), _ptr(g), B,
                                    ctypes.byref(o), _ptr(stats), _stream())
        self._check(st, "bz_cell_solve")
        return g, stats

    def cell_fixed_point(self, f_old, inflow_r, eps, dx, mode="pfp", tol=1e-8, max_iter=100, fixed_iters=0,
                         out=None, fallback="fp"):
        import torch

        B = self._field(f_old, "f_old")
        _arg(inflow_r, "inflow_r", f_old.numel(), device=f_old.device)
        _arg(eps, "eps", B, device=f_old.device)
        g = torch.empty_like(f_old) if out is None else _arg(out, "out", f_old.numel(), device=f_old.device)
        stats = self._stats_tensor(B, f_old.device)
        o = self._opts(mode, tol, max_iter, fixed_iters, fallback)
        st = self.lib.bz_cell_fixed_point(self.h, _ptr(f_old), _ptr(inflow_r), _ptr(eps), float(dx), _ptr(g), B,
                                          ctypes.byref(o), _ptr(stats), _stream())
        self._check(st, "bz_cell_fixed_point")
        return g, stats

    def cell_fixed_point_ex(self, f_old, inflow_r, eps, dx=0.0, nu=None, dxs=None, g0=None, mode="pfp", tol=1e-8,
                            max_iter=100, fixed_iters=0, out=None, fallback="fp"):
        """bz_cell_fixed_point_ex: the cell update with optional per-cell penalty
        frequency nu [B], per-cell widths dxs [B] and initial guesses g0 [B, K]."""
        import torch

        B = self._field(f_old, "f_old")
        _arg(inflow_r, "inflow_r", f_old.numel(), device=f_old.device)
        _arg(eps, "eps", B, device=f_old.device)
        _arg(nu, "nu", B, device=f_old.device, optional=True)
        _arg(dxs, "dxs", B, device=f_old.device, optional=True)
        _arg(g0, "g0", f_old.numel(), device=f_old.device, optional=True)
        g = torch.empty_like(f_old) if out is None else _arg(out, "out", f_old.numel(), device=f_old.device)
        stats = self._stats_tensor(B, f_old.device)
        o = self._opts(mode, tol, max_iter, fixed_iters, fallback)
        st = self.lib.bz_cell_fixed_point_ex(self.h, _ptr(f_old), _ptr(inflow_r), _ptr(eps), _ptr(nu), float(dx),
                                             _ptr(dxs), _ptr(g0), _ptr(g), B, ctypes.byref(o), _ptr(stats), _stream())
        self._check(st, "bz_cell_fixed_point_ex")
        return g, stats

    def cell_fixed_point_learned(self, mlp, f_old, inflow_r, eps, dx, mode="pfp", tol=1e-8, max_iter=100,
                                 fixed_iters=0, out=None):
        import torch

        B = self._field(f_old, "f_old")
        _arg(inflow_r, "inflow_r", f_old.numel(), device=f_old.device)
        _arg(eps, "eps", B, device=f_old.device)
        if mlp.n_in != self.K + 6 or mlp.n_out != self.K:
            raise BZError(f"the network must map K + 6 = {self.K + 6} inputs to K = {self.K} outputs")
        g = torch.empty_like(f_old) if out is None else _arg(out, "out", f_old.numel(), device=f_old.device)
        stats = self._stats_tensor(B, f_old.device)
        o = self._opts(mode, tol, max_iter, fixed_iters)
        st = self.lib.bz_cell_fixed_point_learned(self.h, mlp.h, _ptr(f_old), _ptr(inflow_r), _ptr(eps), float(dx),
                                                  _ptr(g), B, ctypes.byref(o), _ptr(stats), _stream())
        self._check(st, "bz_cell_fixed_point_learned")
        return g, stats

    def features(self, inflow_r, theta, eps, dx):
        import torch

        B = self._field(inflow_r, "inflow_r")
        _arg(theta, "theta", B * (self.d + 2), device=inflow_r.device)
        _arg(eps, "eps", B, device=inflow_r.device)
        X = torch.empty((B, self.K + (6 if self.d == 3 else 5)), dtype=torch.float32, device=inflow_r.device)
        self._check(self.lib.bz_mlp_features(self.h, _ptr(inflow_r), _ptr(theta), _ptr(eps), float(dx), _ptr(X), B,
                                             _stream()), "bz_mlp_features")
        return X

    def set_plan(self, pair_waves: int = 0, chunk_cells: int = 0, acc_nodes: int = 0):
        """bz_set_plan: launch plan of the collision pipeline (0 = default)."""
        p = bz_plan(pair_waves, chunk_cells, acc_nodes)
        self._check(self.lib.bz_set_plan(self.h, ctypes.byref(p)), "bz_set_plan")

    def get_plan(self):
        p = bz_plan()
        self._check(self.lib.bz_get_plan(self.h, ctypes.byref(p)), "bz_get_plan")
        return {"pair_waves": p.pair_waves, "chunk_cells": p.chunk_cells, "acc_nodes": p.acc_nodes}

    def tune(self, f, corrected: bool = True, conserve: str | None = None, reps: int = 2):
        """bz_tune: time bz_eval_Q on f under every candidate plan, keep and cache
        the fastest.  Returns the report as a list of (plan, ms) and the best index."""
        B = self._field(f, "f")
        flags = (BZ_Q_CORRECTED if corrected else 0) | {None: 0, "mass": BZ_Q_MASS, "all": BZ_Q_CONSERVE}[conserve]
        rep = bz_tune_report()
        self._check(self.lib.bz_tune(self.h, _ptr(f), B, flags, reps, ctypes.byref(rep), _stream()), "bz_tune")
        cands = [({"pair_waves": rep.plan[i].pair_waves, "chunk_cells": rep.plan[i].chunk_cells,
                   "acc_nodes": rep.plan[i].acc_nodes}, rep.ms[i]) for i in range(rep.n)]
        return {"candidates": cands, "best": rep.best, "plan": cands[rep.best][0]}

    def profile_enable(self, on: bool = True):
        self._check(self.lib.bz_profile_enable(self.h, 1 if on else 0), "bz_profile_enable")

    def profile_get(self):
        info = bz_profile_info()
        self._check(self.lib.bz_profile_get(self.h, ctypes.byref(info)), "bz_profile_get")
        return {"launches": info.launches, "total_ms": info.total_ms, "flops": info.flops}


# Multigrid parameters of tab. mg (Section 3.4): (spatial dimension, order of
# the scheme) -> (coarsest grid in cells per direction, pre-smoothing steps,
# post-smoothing steps) of the FAS V-cycle.
MG_PARAMS = {(1, 1): (4, 1, 1), (1, 2): (8, 5, 1), (2, 1): (5, 1, 1), (2, 2): (5, 5, 1)}


def mg_params(dim: int, order: int) -> dict:
    """The V-cycle keywords (coarsest, nu1, nu2) of tab. mg for a 1D (slab) or
    2D (cavity) problem with a first- or second-order scheme."""
    c, n1, n2 = MG_PARAMS[(dim, order)]
    return {"coarsest": c, "nu1": n1, "nu2": n2}


class Slab:
    """A set of 1D slab instances sharing one context (bz_slab).

    ``instances`` is a list of dicts with keys xL, xR, nx, eps, T_L, T_R, U_L, U_R,
    mass, and optionally bc_L / bc_R ("wall" or "inflow") with rho_L / rho_R.  ``f`` is a float64 device tensor [sum nx, K] that the slab reads and
    updates in place (borrowed for the slab's lifetime).  ``order`` is the
    spatial order (1, or 2 for the linear reconstruction).  ``mode`` is the
    visit's iteration: "pfp", "fp", or "si" (the source iteration, BGK only)."""

    def __init__(self, ctx: Context, instances, f, collision: str = "binary", bgk_nu: float = 0.0,
                 mode="pfp", tol=1e-8, max_iter=100, fixed_iters=0, order: int = 1, limiter: str = "none",
                 fallback: str = "fp"):
        self.ctx = ctx
        self.f = f
        n = len(instances)
        arr = (bz_slab_instance * n)()
        for i, d in enumerate(instances):
            arr[i].xL, arr[i].xR, arr[i].nx, arr[i].eps = d.get("xL", 0.0), d.get("xR", 1.0), d["nx"], d["eps"]
            arr[i].T_L, arr[i].T_R, arr[i].mass = d.get("T_L", 1.0), d.get("T_R", 2.0), d.get("mass", 1.0)
            for a in range(3):
                arr[i].U_L[a] = d.get("U_L", (0.0, 0.0, 0.0))[a]
                arr[i].U_R[a] = d.get("U_R", (0.0, 0.0, 0.0))[a]
            kinds = {"wall": BZ_BC_WALL, "inflow": BZ_BC_INFLOW}
            arr[i].bc_L, arr[i].bc_R = kinds[d.get("bc_L", "wall")], kinds[d.get("bc_R", "wall")]
            arr[i].rho_L, arr[i].rho_R = d.get("rho_L", 1.0), d.get("rho_R", 1.0)
        total = sum(d["nx"] for d in instances)
        ctx._field(f, "f")
        if f.numel() != total * ctx.K:
            raise BZError("f must hold sum(nx) cells")
        self._arr = arr
        desc = bz_slab_desc(n, arr, _COLLISIONS[collision], bgk_nu,
                            Context._opts(mode, tol, max_iter, fixed_iters, fallback), ctypes.c_void_p(f.data_ptr()),
                            order, _LIMITERS[limiter])
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.bz_slab_create(ctx.h, ctypes.byref(desc), ctypes.byref(h)), "bz_slab_create")
        self.h = h
        self.n = n

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.bz_slab_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stats(st):
        return {"n_iters": st.n_iters, "inner_iters": st.inner_iters, "visits": st.visits, "fallbacks": st.fallbacks,
                "learned": st.learned}

    def inflow(self, out=None):
        """bz_slab_inflow: the transport part of eq. r of every cell of the current
        iterate, both neighbours (and ghosts) from that iterate; [sum nx, K]."""
        import torch

        T = torch.empty_like(self.f) if out is None else _arg(out, "out", self.f.numel(), device=self.f.device)
        self.ctx._check(self.ctx.lib.bz_slab_inflow(self.ctx.h, self.h, _ptr(T), _stream()), "bz_slab_inflow")
        return T

    def attach_warmstart(self, mlp):
        """bz_ws_attach: start visits from the network's guess where its inner
        residual is the smaller (None detaches).  Keeps a reference to mlp."""
        if mlp is not None and (mlp.n_in != self.ctx.K + 6 or mlp.n_out != self.ctx.K):
            raise BZError(f"the network must map K + 6 = {self.ctx.K + 6} inputs to K = {self.ctx.K} outputs")
        self.ctx._check(self.ctx.lib.bz_ws_attach(self.h, mlp.h if mlp is not None else None), "bz_ws_attach")
        self._ws = mlp

    def sweep(self, n_iters: int = 1):
        """n_iters SGS iterations; returns (residuals per instance, stats)."""
        res = (ctypes.c_double * self.n)()
        st = bz_sweep_stats()
        self.ctx._check(self.ctx.lib.bz_sgs_sweep(self.ctx.h, self.h, n_iters, res, ctypes.byref(st), _stream()),
                        "bz_sgs_sweep")
        return list(res), self._stats(st)

    def residual(self):
        res = (ctypes.c_double * self.n)()
        self.ctx._check(self.ctx.lib.bz_outer_residual(self.ctx.h, self.h, res, _stream()), "bz_outer_residual")
        return list(res)

    def vcycle(self, n_cycles: int = 1, coarsest: int = 4, nu1: int = 1, nu2: int = 1, coarse_iters: int = 20,
               tol: float = 1e-5, fixed_cycle: bool = False):
        """n_cycles FAS V-cycles; fixed_cycle: no residual-based exits (the
        cycle capture_vcycles records)."""
        o = bz_mg_opts(coarsest, nu1, nu2, coarse_iters, tol, 1 if fixed_cycle else 0)
        res = (ctypes.c_double * self.n)()
        st = bz_sweep_stats()
        self.ctx._check(self.ctx.lib.bz_multigrid_vcycle(self.ctx.h, self.h, ctypes.byref(o), n_cycles, res,
                                                         ctypes.byref(st), _stream()), "bz_multigrid_vcycle")
        return list(res), self._stats(st)

    def capture(self, iters: int, with_residual: bool = True) -> "SweepGraph":
        """Capture iters SGS iterations into a replayable HIP graph."""
        return SweepGraph(self, iters, with_residual)

    def capture_vcycles(self, cycles: int, coarsest: int = 4, nu1: int = 1, nu2: int = 1, coarse_iters: int = 20,
                        with_residual: bool = True) -> "SweepGraph":
        """Capture cycles fixed-structure FAS V-cycles (each with the mass
        rescale) into a replayable HIP graph."""
        return SweepGraph(self, cycles, with_residual, mg=bz_mg_opts(coarsest, nu1, nu2, coarse_iters, 0.0, 1))


class Cavity:
    """A 2D cavity on [0, 1]^2 (bz_cavity) on a context with d = 2.

    ``walls`` lists (T, (U_1, U_2)) for the sides x = 0, x = 1, y = 0, y = 1.
    ``uniform_y`` (ny = 1): the slab between two plates, no y transport or walls.
    ``f`` is a float64 device tensor [nx * ny, K] (cell (i, j) at row i * ny + j)
    that the cavity reads and updates in place (borrowed for its lifetime)."""

    def __init__(self, ctx: Context, nx: int, ny: int, eps: float, walls, f, mass: float = 1.0,
                 collision: str = "binary", bgk_nu: float = 0.0, mode="pfp", tol=1e-8, max_iter=100,
                 fixed_iters=0, order: int = 1, uniform_y: bool = False, fallback: str = "fp",
                 limiter: str = "none"):
        self.ctx = ctx
        self.f = f
        ctx._field(f, "f")
        if f.numel() != nx * ny * ctx.K:
            raise BZError("f must hold nx * ny cells")
        wl = (bz_wall * 4)()
        for s_, (T, U) in enumerate(walls):
            wl[s_].T = T
            wl[s_].U[0], wl[s_].U[1] = U
        desc = bz_cavity_desc(nx, ny, eps, wl, mass, _COLLISIONS[collision], bgk_nu,
                              Context._opts(mode, tol, max_iter, fixed_iters, fallback), ctypes.c_void_p(f.data_ptr()),
                              order,
                              1 if uniform_y else 0, _LIMITERS[limiter])
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.bz_cavity_create(ctx.h, ctypes.byref(desc), ctypes.byref(h)), "bz_cavity_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.bz_cavity_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n_iters: int = 1, residual: bool = True):
        """n_iters SGS iterations (four scans each); returns (outer residual or None, stats)."""
        res = ctypes.c_double(0.0)
        st = bz_sweep_stats()
        self.ctx._check(self.ctx.lib.bz_cavity_sweep(self.ctx.h, self.h, n_iters,
                                                     ctypes.byref(res) if residual else None, ctypes.byref(st),
                                                     _stream()), "bz_cavity_sweep")
        return (res.value if residual else None), Slab._stats(st)

    def vcycle(self, n_cycles: int = 1, coarsest: int = 5, nu1: int = 1, nu2: int = 1, coarse_iters: int = 20,
               tol: float = 1e-5):
        """n_cycles FAS V-cycles (each followed by the mass rescale); returns (residual, stats).
        The defaults are tab. mg's for a first-order 2D scheme (coarsest 5 x 5)."""
        o = bz_mg_opts(coarsest, nu1, nu2, coarse_iters, tol)
        res = ctypes.c_double(0.0)
        st = bz_sweep_stats()
        self.ctx._check(self.ctx.lib.bz_cavity_vcycle(self.ctx.h, self.h, ctypes.byref(o), n_cycles, ctypes.byref(res),
                                                      ctypes.byref(st), _stream()), "bz_cavity_vcycle")
        return res.value, Slab._stats(st)

    def residual(self) -> float:
        res = ctypes.c_double(0.0)
        self.ctx._check(self.ctx.lib.bz_cavity_residual(self.ctx.h, self.h, ctypes.byref(res), _stream()),
                        "bz_cavity_residual")
        return res.value

    def inflow(self, out=None):
        """bz_cavity_inflow: the transport part of every cell's right-hand side of
        the current field, all neighbours (and wall ghosts) from that field; [nx * ny, K]."""
        import torch

        T = torch.empty_like(self.f) if out is None else _arg(out, "out", self.f.numel(), device=self.f.device)
        self.ctx._check(self.ctx.lib.bz_cavity_inflow(self.ctx.h, self.h, _ptr(T), _stream()), "bz_cavity_inflow")
        return T

    def attach_warmstart(self, mlp):
        """bz_cavity_ws_attach: start visits from the network's guess where its inner
        residual is the smaller (None detaches).  Keeps a reference to mlp."""
        if mlp is not None and (mlp.n_in != self.ctx.K + 5 or mlp.n_out != self.ctx.K):
            raise BZError(f"the network must map K + 5 = {self.ctx.K + 5} inputs to K = {self.ctx.K} outputs")
        self.ctx._check(self.ctx.lib.bz_cavity_ws_attach(self.h, mlp.h if mlp is not None else None),
                        "bz_cavity_ws_attach")
        self._ws = mlp


class SweepGraph:
    """iters SGS iterations, or iters fixed-structure V-cycles (mg given), and
    optionally the outer residual, of a Slab captured into a HIP graph
    (bz_graph_capture_sweeps / bz_graph_capture_vcycles), replayed on a
    dedicated stream of default priority that is ordered after the caller's
    current stream."""

    def __init__(self, slab: "Slab", iters: int, with_residual: bool = True, mg=None):
        import torch

        self.slab = slab
        self.ctx = slab.ctx
        self.iters = iters
        self.with_residual = with_residual
        self.stream = torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if mg is None:
            self.ctx._check(self.ctx.lib.bz_graph_capture_sweeps(self.ctx.h, slab.h, iters, 1 if with_residual else 0,
                                                                 sp, ctypes.byref(h)), "bz_graph_capture_sweeps")
        else:
            self._mg = mg
            self.ctx._check(self.ctx.lib.bz_graph_capture_vcycles(self.ctx.h, slab.h, ctypes.byref(mg), iters,
                                                                  1 if with_residual else 0, sp, ctypes.byref(h)),
                            "bz_graph_capture_vcycles")
        self.h = h

    def launch(self):
        """One replay; returns (per-instance residuals or None, stats)."""
        import torch

        self.stream.wait_stream(torch.cuda.current_stream())
        res = (ctypes.c_double * self.slab.n)() if self.with_residual else None
        st = bz_sweep_stats()
        self.ctx._check(self.ctx.lib.bz_graph_launch(self.h, res, ctypes.byref(st),
                                                     ctypes.c_void_p(self.stream.cuda_stream)), "bz_graph_launch")
        torch.cuda.current_stream().wait_stream(self.stream)
        return (list(res) if res is not None else None), self.slab._stats(st)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.bz_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The warm-start network (bz_mlp): FP32 parameters on the device."""

    def __init__(self, ctx: Context, n_in: int, hidden: int, n_out: int, seed: int = 0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.bz_mlp_create(ctx.h, n_in, hidden, n_out, seed, ctypes.byref(h)), "bz_mlp_create")
        self.h = h
        self.n_in, self.hidden, self.n_out = n_in, hidden, n_out
        self.n_params = int(ctx.lib.bz_mlp_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.bz_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np

        buf = np.empty(self.n_params, dtype=np.float32)
        self.ctx._check(self.ctx.lib.bz_mlp_get_params(self.h, buf.ctypes.data, self.n_params), "bz_mlp_get_params")
        return buf

    def set_params(self, p):
        import numpy as np

        buf = np.ascontiguousarray(p, dtype=np.float32)
        self.ctx._check(self.ctx.lib.bz_mlp_set_params(self.h, buf.ctypes.data, self.n_params), "bz_mlp_set_params")

    def set_output_scale(self, s: float):
        self.ctx._check(self.ctx.lib.bz_mlp_set_output_scale(self.h, float(s)), "bz_mlp_set_output_scale")

    def _xt(self, X, T=None):
        B = X.shape[0] if X.dim() == 2 else -1
        if B < 0:
            raise BZError("X must be [batch, n_in]")
        _arg(X, "X", B * self.n_in, dtype="float32")
        if T is not None:
            _arg(T, "T", B * self.n_out, dtype="float32", device=X.device)
        return B

    def forward(self, X, bf16: bool = False):
        import torch

        B = self._xt(X)
        Y = torch.empty((B, self.n_out), dtype=torch.float32, device=X.device)
        self.ctx._check(self.ctx.lib.bz_mlp_forward(self.h, _ptr(X), _ptr(Y), B, 1 if bf16 else 0, _stream()),
                        "bz_mlp_forward")
        return Y

    def grad(self, X, T):
        import torch

        self._xt(X, T)
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        self.ctx._check(self.ctx.lib.bz_mlp_grad(self.h, _ptr(X), _ptr(T), X.shape[0], _ptr(g), ctypes.byref(loss),
                                                 _stream()), "bz_mlp_grad")
        return loss.value, g

    def train_step(self, X, T, lr: float, want_loss: bool = False):
        self._xt(X, T)
        loss = ctypes.c_double()
        self.ctx._check(self.ctx.lib.bz_mlp_train_step(self.h, _ptr(X), _ptr(T), X.shape[0], float(lr),
                                                       ctypes.byref(loss) if want_loss else None, _stream()),
                        "bz_mlp_train_step")
        return loss.value if want_loss else None
