"""ctypes binding of libslim.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers, host lists to int32 arrays, and status codes to
exceptions.  It never falls back to a CPU implementation: if the library is
missing it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch  # loads the HIP runtime first, so libslim binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libslim.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "slim.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(_HERE), "include", "slim_cnn.h"),
           os.path.join(os.path.dirname(_HERE), "include", "slim3d.h")]

SLIM_OK, SLIM_EINVAL, SLIM_ENOMEM, SLIM_EDEVICE, SLIM_ENUMERIC, SLIM_ENOTCONV, SLIM_ESTATE = range(7)
PREC = {"fp32": 0, "bf16": 1}
GRAM = {"auto": 0, "chol": 1, "pcg": 2, "jacobi": 3}


class SlimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"slim status {status}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("n_slices", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("angles_per_block", ctypes.c_int), ("precision", ctypes.c_int),
                ("gram_mode", ctypes.c_int), ("chol_max_p", ctypes.c_int),
                ("pcg_max_iter", ctypes.c_int), ("pcg_tol", ctypes.c_double),
                ("check_every", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("use_graph", ctypes.c_int),
                ("damping_ramp", ctypes.c_int), ("tikhonov", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("step_norm", ctypes.c_double), ("x_norm", ctypes.c_double),
                ("err_norm", ctypes.c_double), ("k", ctypes.c_int), ("pcg_iters", ctypes.c_int),
                ("pcg_relres", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("epochs", ctypes.c_int), ("converged", ctypes.c_int),
                ("rho_last", ctypes.c_double), ("err_last", ctypes.c_double),
                ("pcg_iters", ctypes.c_int)]


class Tune(ctypes.Structure):
    _fields_ = [("fwd_bt", ctypes.c_int), ("fwd_items", ctypes.c_int), ("fwd_slots", ctypes.c_int),
                ("back_bt", ctypes.c_int)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("chosen", Tune), ("fwd_us", ctypes.c_double), ("back_us", ctypes.c_double),
                ("fwd_default_us", ctypes.c_double), ("back_default_us", ctypes.c_double),
                ("candidates", ctypes.c_int), ("cached", ctypes.c_int)]


class CnnDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("levels", ctypes.c_int), ("channels", ctypes.c_int * 4),
                ("max_batch", ctypes.c_int), ("in_scale", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libslim.so (built by ``build()``); raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "slim_default_opts": (I, [ctypes.POINTER(Opts)]),
        "slim_init": (I, [ctypes.POINTER(P), ctypes.POINTER(Grid), I, ctypes.POINTER(D), I, I, D,
                          ctypes.POINTER(Opts)]),
        "slim_set_data": (I, [P, P, P, P]),
        "slim_step": (I, [P, i32p, I, ctypes.POINTER(StepInfo)]),
        "slim_set_lambda": (I, [P, D]),
        "slim_step_data": (I, [P, i32p, I, P, ctypes.POINTER(StepInfo)]),
        "slim_solve": (I, [P, P, P, P, D, I, ctypes.POINTER(SolveInfo)]),
        "slim_project": (I, [P, i32p, I, P, P]),
        "slim_project_noalloc": (I, [P, i32p, I, P, P]),
        "slim_backproject": (I, [P, i32p, I, P, P]),
        "slim_gram": (I, [P, i32p, I, i32p, I, P]),
        "slim_get_state": (I, [P, P, ctypes.POINTER(ctypes.c_int64)]),
        "slim_set_state": (I, [P, P, ctypes.c_int64]),
        "slim_slice_norms": (I, [P, ctypes.POINTER(D), I]),
        "slim_profile": (I, [P, I]),
        "slim_kernel_stats": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64)]),
        "slim_data_backprojection": (I, [P, i32p, I, P]),
        "slim_autotune": (I, [P, I, I, ctypes.POINTER(TuneInfo)]),
        "slim_group_create": (I, [ctypes.POINTER(P), ctypes.POINTER(P), I]),
        "slim_group_step": (I, [P, i32p, I, ctypes.POINTER(StepInfo)]),
        "slim_group_destroy": (None, [P]),
        "slim_group_set_shared": (I, [P, I]),
        "slim_set_tune": (I, [P, ctypes.POINTER(Tune)]),
        "slim_get_tune": (I, [P, ctypes.POINTER(Tune)]),
        "slim_warmstart": (I, [P, P, i32p, I, P, ctypes.POINTER(I)]),
        "slim_cnn_create": (I, [ctypes.POINTER(P), ctypes.POINTER(CnnDesc)]),
        "slim_cnn_num_params": (ctypes.c_int64, [P]),
        "slim_cnn_set_params": (I, [P, P, ctypes.c_int64]),
        "slim_cnn_get_params": (I, [P, P, ctypes.c_int64]),
        "slim_cnn_forward": (I, [P, P, P, I]),
        "slim_cnn_loss_grad": (I, [P, P, P, I, ctypes.POINTER(D), P]),
        "slim_cnn_adam": (I, [P, D, D, D, D]),
        "slim_cnn_forward_flops": (D, [P]),
        "slim_cnn_destroy": (None, [P]),
        "slim_destroy": (None, [P]),
        "slim3d_init": (I, [ctypes.POINTER(P), I, I, ctypes.POINTER(D), I, I, D,
                            ctypes.POINTER(Opts)]),
        "slim3d_set_data": (I, [P, P, P, P]),
        "slim3d_step": (I, [P, i32p, I, ctypes.POINTER(StepInfo)]),
        "slim3d_project": (I, [P, i32p, I, P, P]),
        "slim3d_backproject": (I, [P, i32p, I, P, P]),
        "slim3d_profile": (I, [P, I]),
        "slim3d_kernel_stats": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64)]),
        "slim3d_destroy": (None, [P]),
        "slim_strerror": (ctypes.c_char_p, [I]),
        "slim_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols() -> list[str]:
    """Names of the functions declared in include/slim.h, slim_cnn.h and
    slim3d.h."""
    txt = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"\b(slim(?:3d)?_[a-z_]+)\s*\(", txt)))


def _check(st: int):
    if st != SLIM_OK:
        msg = load().slim_last_error().decode()
        raise SlimError(st, msg or load().slim_strerror(st).decode())


def _ids(ids) -> tuple:
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.int32).reshape(-1))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(a.size)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Slim:
    """One slimLS context bound to the current device and torch stream."""

    def __init__(self, N: int, n_angles: int, n_rays: int | None = None, r: int = 0,
                 lam: float = 1e-2, n_slices: int = 1, angles_per_block: int = 1,
                 precision: str = "fp32", gram_mode: str = "auto", chol_max_p: int = 8192,
                 pcg_max_iter: int = 1000, pcg_tol: float = 1e-6, check_every: int = 1,
                 seed: int = 0, angles=None, stream=None, use_graph: bool = True,
                 damping_ramp: bool = False, tikhonov: float = 0.0):
        lib = load()
        if n_rays is None:
            n_rays = 2 * int(np.floor(N / np.sqrt(2.0))) + 1
        self.N, self.n_angles, self.R, self.r = int(N), int(n_angles), int(n_rays), int(r)
        self.lam, self.B, self.g = float(lam), int(n_slices), int(angles_per_block)
        self.precision = precision
        o = Opts()
        lib.slim_default_opts(ctypes.byref(o))
        o.angles_per_block = self.g
        o.precision = PREC[precision]
        o.gram_mode = GRAM[gram_mode]
        o.chol_max_p = int(chol_max_p)
        o.pcg_max_iter = int(pcg_max_iter)
        o.pcg_tol = float(pcg_tol)
        o.check_every = int(check_every)
        o.seed = int(seed) & ((1 << 64) - 1)
        o.use_graph = int(bool(use_graph))
        o.damping_ramp = int(bool(damping_ramp))
        o.tikhonov = float(tikhonov)
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        o.stream = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        self.stream = stream
        ang = None
        if angles is not None:
            self._angles = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
            ang = self._angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g = Grid(self.N, self.B)
        h = ctypes.c_void_p()
        _check(lib.slim_init(ctypes.byref(h), ctypes.byref(g), self.n_angles, ang, self.R, self.r,
                             self.lam, ctypes.byref(o)))
        self._h = h
        self._keep = []

    # --- data and iteration ------------------------------------------------
    def _b_dtype(self):
        return torch.bfloat16 if self.precision == "bf16" else torch.float32

    def set_data(self, b, x, x_true=None):
        """Bind b (None: streaming data, see step_data), x and x_true."""
        nb, nx = self.B * self.n_angles * self.R, self.B * self.N * self.N
        for t, n, name in ((b, nb, "b"), (x, nx, "x"), (x_true, nx, "x_true")):
            if t is not None and isinstance(t, torch.Tensor) and t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
        self._keep = [b, x, x_true]
        _check(load().slim_set_data(self._h, _ptr(b, self._b_dtype(), "b"),
                                    _ptr(x, torch.float32, "x"),
                                    _ptr(x_true, torch.float32, "x_true")))

    def step(self, angle_ids, read: bool = True) -> dict | None:
        a, p, n = _ids(angle_ids)
        info = StepInfo()
        _check(load().slim_step(self._h, p, n, ctypes.byref(info) if read else None))
        if not read:
            return None
        return {f: getattr(info, f) for f, _ in StepInfo._fields_}

    def step_data(self, angle_ids, b_block, read: bool = True) -> dict | None:
        """One step with the block's data [n_slices][len(ids)][R] (a contiguous
        tensor on the GPU or in host memory, pinned for an asynchronous copy)."""
        a, p, n = _ids(angle_ids)
        if not isinstance(b_block, torch.Tensor) or not b_block.is_contiguous():
            raise ValueError("b_block must be a contiguous torch tensor")
        if b_block.dtype != self._b_dtype():
            raise TypeError(f"b_block must be {self._b_dtype()}")
        if b_block.numel() != self.B * n * self.R:
            raise ValueError(f"b_block has {b_block.numel()} elements, expected {self.B * n * self.R}")
        # the copy may still be pending after an unread step: hold every block
        # until a step is read back (which synchronises the stream)
        self._blocks = getattr(self, "_blocks", []) + [b_block]
        info = StepInfo()
        _check(load().slim_step_data(self._h, p, n, ctypes.c_void_p(b_block.data_ptr()),
                                     ctypes.byref(info) if read else None))
        if not read:
            return None
        self._blocks = []
        return {f: getattr(info, f) for f, _ in StepInfo._fields_}

    def set_lambda(self, lam: float):
        """Damping lambda = 1/alpha of the following steps."""
        _check(load().slim_set_lambda(self._h, float(lam)))
        self.lam = float(lam)

    def slice_norms(self) -> np.ndarray:
        """[n_slices][3] float64: ||s_k||, ||x_k||, ||x_k - x_true|| of the last
        step read back, slice by slice."""
        out = np.zeros((self.B, 3), dtype=np.float64)
        _check(load().slim_slice_norms(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       self.B))
        return out

    def autotune(self, n_ids: int = 0, force: bool = False) -> dict:
        """Measure projector launch shapes on lists of n_ids angles (0: this
        context's CG window, also the default shape) and keep the fastest;
        returns the chosen shape and the times."""
        ti = TuneInfo()
        _check(load().slim_autotune(self._h, int(n_ids), int(bool(force)), ctypes.byref(ti)))
        out = {f: getattr(ti, f) for f, _ in TuneInfo._fields_ if f != "chosen"}
        out["chosen"] = {f: getattr(ti.chosen, f) for f, _ in Tune._fields_}
        return out

    def set_tune(self, fwd_bt=0, fwd_items=0, fwd_slots=0, back_bt=0):
        t = Tune(fwd_bt, fwd_items, fwd_slots, back_bt)
        _check(load().slim_set_tune(self._h, ctypes.byref(t)))

    def get_tune(self) -> dict:
        t = Tune()
        _check(load().slim_get_tune(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Tune._fields_}

    def data_backprojection(self, angle_ids, out=None):
        """out = A_ids^T b_ids for the bound data, every slice."""
        a, p, n = _ids(angle_ids)
        if out is None:
            shape = (self.B, self.N, self.N) if self.B > 1 else (self.N, self.N)
            out = torch.empty(shape, dtype=torch.float32, device="cuda")
        _check(load().slim_data_backprojection(self._h, p, n, _ptr(out, torch.float32, "out")))
        return out

    def warmstart(self, angle_ids, x0=None, net: "Cnn | None" = None):
        """x0 = net(A_ids^T b_ids) for the bound data (zeros without a usable
        network).  Returns (x0, used_net)."""
        a, p, n = _ids(angle_ids)
        if x0 is None:
            shape = (self.B, self.N, self.N) if self.B > 1 else (self.N, self.N)
            x0 = torch.empty(shape, dtype=torch.float32, device="cuda")
        used = ctypes.c_int(0)
        _check(load().slim_warmstart(self._h, net._h if net is not None else None, p, n,
                                     _ptr(x0, torch.float32, "x0"), ctypes.byref(used)))
        return x0, bool(used.value)

    def solve(self, b, x, x_true=None, tol: float = 1e-2, max_epochs: int = 1) -> dict:
        self._keep = [b, x, x_true]
        info = SolveInfo()
        _check(load().slim_solve(self._h, _ptr(b, self._b_dtype(), "b"),
                                 _ptr(x, torch.float32, "x"),
                                 _ptr(x_true, torch.float32, "x_true"), float(tol),
                                 int(max_epochs), ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in SolveInfo._fields_}

    # --- operators -----------------------------------------------------------
    def project(self, angle_ids, x, out=None):
        a, p, n = _ids(angle_ids)
        if out is None:
            out = torch.empty((self.B, n, self.R) if self.B > 1 else (n, self.R),
                              dtype=torch.float32, device=x.device)
        _check(load().slim_project(self._h, p, n, _ptr(x, torch.float32, "x"),
                                   _ptr(out, torch.float32, "out")))
        return out

    def project_noalloc(self, angle_ids, x, out):
        """slim_project into a caller-given ``out`` through the library's fixed
        scratch (no device allocation in the call)."""
        a, p, n = _ids(angle_ids)
        _check(load().slim_project_noalloc(self._h, p, n, _ptr(x, torch.float32, "x"),
                                           _ptr(out, torch.float32, "out")))
        return out

    def backproject(self, angle_ids, v, out=None):
        a, p, n = _ids(angle_ids)
        if out is None:
            shape = (self.B, self.N, self.N) if self.B > 1 else (self.N, self.N)
            out = torch.empty(shape, dtype=torch.float32, device=v.device)
        _check(load().slim_backproject(self._h, p, n, _ptr(v, torch.float32, "v"),
                                       _ptr(out, torch.float32, "out")))
        return out

    def gram(self, ids_a, ids_b, out=None, device="cuda"):
        a, pa, na = _ids(ids_a)
        b, pb, nb = _ids(ids_b)
        if out is None:
            out = torch.empty((na * self.R, nb * self.R), dtype=torch.float64, device=device)
        _check(load().slim_gram(self._h, pa, na, pb, nb, _ptr(out, torch.float64, "out")))
        return out

    # --- checkpoint ----------------------------------------------------------
    def get_state(self) -> bytes:
        size = ctypes.c_int64(0)
        st = load().slim_get_state(self._h, None, ctypes.byref(size))
        if st not in (SLIM_OK, SLIM_EINVAL):
            _check(st)
        buf = ctypes.create_string_buffer(size.value)
        _check(load().slim_get_state(self._h, buf, ctypes.byref(size)))
        return buf.raw[:size.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(load().slim_set_state(self._h, buf, len(blob)))

    # --- measurement ------------------------------------------------------------
    KINDS = ("cg_forward", "cg_back", "gram", "cholesky", "cg_vector", "residual", "update",
             "cg_forward_reduce")

    def profile(self, on: bool = True):
        _check(load().slim_profile(self._h, int(on)))

    def kernel_stats(self) -> dict:
        out = {}
        for k, name in enumerate(self.KINDS):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_int64(0)
            _check(load().slim_kernel_stats(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = {"total_ms": ms.value, "launches": n.value}
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().slim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_error(**kw) -> int:
    """Status of slim_init for the given arguments (no context kept).

    Used to exercise argument validation, which runs before any device call."""
    lib = load()
    N = kw.get("N", 64)
    o = Opts()
    lib.slim_default_opts(ctypes.byref(o))
    o.angles_per_block = kw.get("angles_per_block", 1)
    o.precision = kw.get("precision", 0)
    o.gram_mode = kw.get("gram_mode", 0)
    o.check_every = kw.get("check_every", 1)
    o.damping_ramp = kw.get("damping_ramp", 0)
    o.tikhonov = kw.get("tikhonov", 0.0)
    g = Grid(N, kw.get("n_slices", 1))
    h = ctypes.c_void_p()
    st = lib.slim_init(ctypes.byref(h), ctypes.byref(g), kw.get("n_angles", 90), None,
                       kw.get("n_rays", 91), kw.get("r", 5), kw.get("lam", 1e-2), ctypes.byref(o))
    if st == SLIM_OK:
        lib.slim_destroy(h)
    return st


class Slim3D:
    """A 3D parallel-beam slimLS context (projection images from arbitrary
    directions) bound to the current device and torch stream."""

    KINDS = {"cg_forward": 0, "cg_back": 1, "cg_vector": 4, "residual": 5, "update": 6}

    def __init__(self, N: int, dirs, n_det: int | None = None, r: int = 0, lam: float = 1e-2,
                 dirs_per_block: int = 1, pcg_max_iter: int = 1000, pcg_tol: float = 1e-6,
                 stream=None, gram_mode: str = "auto"):
        """gram_mode "auto" / "jacobi": CG preconditioned by the inverse Gram
        diagonal; "pcg": plain CG."""
        lib = load()
        self._dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        self.N, self.n_dirs = int(N), int(self._dirs.shape[0])
        self.n_det = int(N if n_det is None else n_det)
        self.r, self.lam, self.g = int(r), float(lam), int(dirs_per_block)
        o = Opts()
        lib.slim_default_opts(ctypes.byref(o))
        o.angles_per_block = self.g
        o.pcg_max_iter = int(pcg_max_iter)
        o.pcg_tol = float(pcg_tol)
        o.gram_mode = GRAM[gram_mode]
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        o.stream = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.slim3d_init(ctypes.byref(h), self.N, self.n_dirs,
                               self._dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               self.n_det, self.r, self.lam, ctypes.byref(o)))
        self._h = h
        self._keep = []

    def set_data(self, b, x, x_true=None):
        nb, nx = self.n_dirs * self.n_det * self.n_det, self.N ** 3
        for t, n, name in ((b, nb, "b"), (x, nx, "x"), (x_true, nx, "x_true")):
            if t is not None and t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
        self._keep = [b, x, x_true]
        _check(load().slim3d_set_data(self._h, _ptr(b, torch.float32, "b"),
                                      _ptr(x, torch.float32, "x"),
                                      _ptr(x_true, torch.float32, "x_true")))

    def step(self, dir_ids, read: bool = True) -> dict | None:
        a, p, n = _ids(dir_ids)
        info = StepInfo()
        _check(load().slim3d_step(self._h, p, n, ctypes.byref(info) if read else None))
        if not read:
            return None
        return {f: getattr(info, f) for f, _ in StepInfo._fields_}

    def project(self, dir_ids, x, out=None):
        a, p, n = _ids(dir_ids)
        if out is None:
            out = torch.empty((n, self.n_det, self.n_det), dtype=torch.float32, device=x.device)
        _check(load().slim3d_project(self._h, p, n, _ptr(x, torch.float32, "x"),
                                     _ptr(out, torch.float32, "out")))
        return out

    def backproject(self, dir_ids, v, out=None):
        a, p, n = _ids(dir_ids)
        if out is None:
            out = torch.empty((self.N, self.N, self.N), dtype=torch.float32, device=v.device)
        _check(load().slim3d_backproject(self._h, p, n, _ptr(v, torch.float32, "v"),
                                         _ptr(out, torch.float32, "out")))
        return out

    def profile(self, on: bool = True):
        _check(load().slim3d_profile(self._h, int(bool(on))))

    def kernel_stats(self) -> dict:
        out = {}
        for name, k in self.KINDS.items():
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(load().slim3d_kernel_stats(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = {"total_ms": ms.value, "launches": n.value}
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().slim3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Contexts of different grid sizes stepped together with the same block
    (include/slim.h, slim_group_*): their CG solves run in shared launches
    (shared=True) or interleaved by one host loop (False, the library's
    default)."""

    def __init__(self, contexts, shared: bool = False):
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        h = ctypes.c_void_p()
        _check(load().slim_group_create(ctypes.byref(h), arr, len(self.contexts)))
        self._h = h
        self.set_shared(shared)

    def set_shared(self, on: bool):
        _check(load().slim_group_set_shared(self._h, int(bool(on))))

    def step(self, angle_ids, read: bool = True):
        a, p, n = _ids(angle_ids)
        infos = (StepInfo * len(self.contexts))() if read else None
        _check(load().slim_group_step(self._h, p, n, infos))
        if not read:
            return None
        return [{f: getattr(i, f) for f, _ in StepInfo._fields_} for i in infos]

    def close(self):
        if getattr(self, "_h", None):
            load().slim_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_layout(channels) -> list[tuple[str, tuple]]:
    """(name, shape) of the packed warm-start parameters, in order: per conv
    layer (forward order) weights [Cout, 3, 3, Cin] then bias [Cout]; then
    head.w [c_1], head.b [1], head.cu [1]."""
    c = list(channels)
    L = len(c)
    layers = [("e1a", c[0], 1), ("e1b", c[0], c[0])]
    for l in range(2, L + 1):
        layers += [(f"e{l}a", c[l - 1], c[l - 2]), (f"e{l}b", c[l - 1], c[l - 1])]
    for l in range(L - 1, 0, -1):
        layers += [(f"u{l}", c[l - 1], c[l]), (f"d{l}a", c[l - 1], 2 * c[l - 1]),
                   (f"d{l}b", c[l - 1], c[l - 1])]
    out = []
    for name, co, ci in layers:
        out += [(name + ".w", (co, 3, 3, ci)), (name + ".b", (co,))]
    return out + [("head.w", (c[0],)), ("head.b", (1,)), ("head.cu", (1,))]


class Cnn:
    """The warm-start U-Net (include/slim_cnn.h) on the current device and
    torch stream."""

    def __init__(self, N: int, channels=(32, 64, 128, 256), max_batch: int = 8,
                 in_scale: float = 1.0, stream=None):
        lib = load()
        self.N, self.channels, self.max_batch = int(N), tuple(int(c) for c in channels), int(max_batch)
        self.in_scale = float(in_scale)
        d = CnnDesc()
        d.N = self.N
        d.levels = len(self.channels)
        for i, c in enumerate(self.channels[:4]):
            d.channels[i] = c
        d.max_batch = self.max_batch
        d.in_scale = self.in_scale
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        d.stream = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        h = ctypes.c_void_p()
        _check(lib.slim_cnn_create(ctypes.byref(h), ctypes.byref(d)))
        self._h = h
        self.n_params = int(lib.slim_cnn_num_params(h))
        self.layout = cnn_layout(self.channels)

    def pack(self, params: dict) -> np.ndarray:
        return np.concatenate([np.asarray(params[k], np.float32).reshape(-1)
                               for k, _ in self.layout])

    def unpack(self, vec) -> dict:
        out, o = {}, 0
        for k, shape in self.layout:
            n = int(np.prod(shape))
            out[k] = np.asarray(vec[o:o + n]).reshape(shape)
            o += n
        return out

    def set_params(self, params):
        v = self.pack(params) if isinstance(params, dict) else np.asarray(params, np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(load().slim_cnn_set_params(self._h, v.ctypes.data_as(ctypes.c_void_p), v.size))

    def get_params(self) -> np.ndarray:
        v = np.empty(self.n_params, dtype=np.float32)
        _check(load().slim_cnn_get_params(self._h, v.ctypes.data_as(ctypes.c_void_p), v.size))
        return v

    def forward(self, u, x0=None):
        B = u.shape[0]
        if x0 is None:
            x0 = torch.empty_like(u)
        _check(load().slim_cnn_forward(self._h, _ptr(u, torch.float32, "u"),
                                       _ptr(x0, torch.float32, "x0"), int(B)))
        return x0

    def loss_grad(self, u, target, want_grad: bool = False):
        """(loss, gradient as a packed float32 vector or None)."""
        loss = ctypes.c_double(0.0)
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _check(load().slim_cnn_loss_grad(self._h, _ptr(u, torch.float32, "u"),
                                         _ptr(target, torch.float32, "target"), int(u.shape[0]),
                                         ctypes.byref(loss),
                                         g.ctypes.data_as(ctypes.c_void_p) if want_grad else None))
        return loss.value, g

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(load().slim_cnn_adam(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def forward_flops(self) -> float:
        return float(load().slim_cnn_forward_flops(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load().slim_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_create_error(**kw) -> int:
    """Status of slim_cnn_create for the given description (argument checks
    run before any device call)."""
    lib = load()
    d = CnnDesc()
    d.N = kw.get("N", 64)
    ch = kw.get("channels", (32, 64))
    d.levels = kw.get("levels", len(ch))
    for i, c in enumerate(list(ch)[:4]):
        d.channels[i] = c
    d.max_batch = kw.get("max_batch", 1)
    d.in_scale = kw.get("in_scale", 1.0)
    h = ctypes.c_void_p()
    st = lib.slim_cnn_create(ctypes.byref(h), ctypes.byref(d))
    if st == SLIM_OK:
        lib.slim_cnn_destroy(h)
    return st
