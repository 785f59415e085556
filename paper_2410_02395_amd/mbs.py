"""ctypes binding of the C ABI declared in ``include/mbs.h``.

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch provides device memory (complex64 tensors) and the HIP stream.  The
library is loaded from this package directory; if it is missing the import of
``Plan`` raises -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch  # noqa: F401  (loads the HIP runtime torch was built with before libmbs)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MBS_LIBRARY", os.path.join(PKG, "libmbs.so"))

EXPORTS = (
    "mbs_plan_bytes", "mbs_plan_create", "mbs_plan_destroy", "mbs_set_medium", "mbs_solve",
    "mbs_solve_async", "mbs_poll", "mbs_residual", "mbs_residual_history", "mbs_timing_read",
    "mbs_strerror",
)

MBS_OK = 0
MBS_EINVAL = -1
MBS_ENOMEM = -2
MBS_EGAIN = -3
MBS_EDEGENERATE = -4
MBS_ENONFINITE = -5
MBS_EDIVERGED = -6
MBS_ESTATE = -7
MBS_EBUSY = -8
MBS_EHIP = -9
MBS_EUNSUPPORTED = -10

MBS_KB_FROM_K0 = 0x1
MBS_X0_GIVEN = 0x2
MBS_NO_GRAPH = 0x4
MBS_TIMING = 0x8
MBS_NO_FUSION = 0x10

# kernel kinds of mbs_timing_read, in order (with the fused z pass, "z_fwd" covers only the
# x/y edge-slab lines, "z_inv" also forms and transforms the next w, "face" finishes the
# edge-slab lines; "yxy_slabs" is the y, x and inverse-y passes run slab by slab)
KERNEL_KINDS = ("z_fwd", "y_fwd", "x_green", "y_inv", "z_inv", "edge_corr", "face", "reduce", "yxy_slabs")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int64 * 3),
        ("split", ctypes.c_int32 * 3),
        ("periodic", ctypes.c_int32 * 3),
        ("t", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("check_every", ctypes.c_int32),
        ("activation", ctypes.c_double),
        ("zblock", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Ramp(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32 * 3), ("im_n2_max", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("kb2", ctypes.c_double),
        ("c_imag", ctypes.c_double),
        ("K", ctypes.c_double),
        ("normC", ctypes.c_double),
        ("rho_ref", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("subdomain_iterations", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MBSError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2410_02395_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.mbs_plan_bytes.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_size_t)]
    lib.mbs_plan_create.argtypes = [ctypes.POINTER(PlanDesc), P, ctypes.POINTER(P)]
    lib.mbs_plan_destroy.argtypes = [P]
    lib.mbs_set_medium.argtypes = [P, I32, P, D, ctypes.POINTER(Ramp)]
    lib.mbs_solve.argtypes = [P, I32, P, D, I32, P, ctypes.POINTER(Result)]
    lib.mbs_solve_async.argtypes = [P, I32, P, D, I32, P]
    lib.mbs_poll.argtypes = [P, I32, ctypes.POINTER(Result)]
    lib.mbs_residual.argtypes = [P, I32, P, ctypes.POINTER(D)]
    lib.mbs_residual_history.argtypes = [P, I32, ctypes.POINTER(D), I32, ctypes.POINTER(I32)]
    lib.mbs_timing_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64), I32, I32]
    lib.mbs_strerror.argtypes = [I32]
    lib.mbs_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "mbs_strerror":
            getattr(lib, name).restype = I32
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load_library().mbs_strerror(int(status)).decode()


def _check(status: int, what: str):
    if status != MBS_OK:
        raise MBSError(status, what)


def make_desc(shape, split=(1, 1, 1), periodic=(1, 1, 1), t=8, max_batch=1, alpha=0.75,
              flags=0, check_every=0, activation=0.0, zblock=0) -> PlanDesc:
    d = PlanDesc()
    for k in range(3):
        d.shape[k] = int(shape[k])
        d.split[k] = int(split[k])
        d.periodic[k] = int(periodic[k])
    d.t = int(t)
    d.max_batch = int(max_batch)
    d.alpha = float(alpha)
    d.flags = int(flags)
    d.check_every = int(check_every)
    d.activation = float(activation)
    d.zblock = int(zblock)
    d.reserved = 0
    return d


def plan_bytes(shape, split=(1, 1, 1), periodic=(1, 1, 1), t=8, max_batch=1, alpha=0.75,
               flags=0, check_every=0, activation=0.0, zblock=0) -> int:
    lib = load_library()
    out = ctypes.c_size_t(0)
    _check(lib.mbs_plan_bytes(ctypes.byref(make_desc(shape, split, periodic, t, max_batch, alpha,
                                                     flags, check_every, activation, zblock)),
                              ctypes.byref(out)),
           "mbs_plan_bytes")
    return int(out.value)


def _dev_ptr(x: torch.Tensor, shape, name: str) -> int:
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError(f"{name} must be a complex64 CUDA tensor")
    if tuple(x.shape) != tuple(shape) or not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")
    return x.data_ptr()


class Plan:
    """One solver plan (grid, decomposition, slots) on the current device."""

    def __init__(self, shape, split=(1, 1, 1), periodic=(1, 1, 1), t=8, max_batch=1, alpha=0.75,
                 flags=0, check_every=0, stream: Optional[torch.cuda.Stream] = None, activation=0.0,
                 zblock=0):
        self._lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.split = tuple(int(s) for s in split)
        self.periodic = tuple(int(s) for s in periodic)
        self.t = int(t)
        self.max_batch = int(max_batch)
        self.alpha = float(alpha)
        self.flags = int(flags)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.activation = float(activation)
        self._desc = make_desc(shape, split, periodic, t, max_batch, alpha, flags, check_every, activation,
                               zblock)
        h = ctypes.c_void_p(0)
        _check(self._lib.mbs_plan_create(ctypes.byref(self._desc), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)), "mbs_plan_create")
        self._h = h
        self._keep = {}
        self.progress = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mbs_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ---------------------------------------------------------------
    def set_medium(self, slot: int, n: torch.Tensor, k0: float,
                   ramp_width: Sequence[int] = (0, 0, 0), ramp_max: float = 0.0):
        r = Ramp()
        for k in range(3):
            r.width[k] = int(ramp_width[k])
        r.im_n2_max = float(ramp_max)
        _check(self._lib.mbs_set_medium(self._h, int(slot), ctypes.c_void_p(_dev_ptr(n, self.shape, "n")),
                                        float(k0), ctypes.byref(r)), "mbs_set_medium")

    def solve(self, slot: int, S: torch.Tensor, tol: float, max_iter: int,
              out: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None):
        """Blocking solve; returns (field, result dict).  ``x0`` requires a plan
        created with MBS_X0_GIVEN (the field buffer then starts as x0)."""
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=S.device)
        if x0 is not None:
            if not (self.flags & MBS_X0_GIVEN):
                raise ValueError("x0 needs a plan created with MBS_X0_GIVEN")
            out.copy_(x0)
        res = Result()
        st = self._lib.mbs_solve(self._h, int(slot), ctypes.c_void_p(_dev_ptr(S, self.shape, "S")), float(tol),
                                 int(max_iter), ctypes.c_void_p(_dev_ptr(out, self.shape, "out")), ctypes.byref(res))
        _check(st, "mbs_solve")
        return out, res.as_dict()

    def solve_async(self, slot: int, S: torch.Tensor, tol: float, max_iter: int, out: torch.Tensor):
        _check(self._lib.mbs_solve_async(self._h, int(slot), ctypes.c_void_p(_dev_ptr(S, self.shape, "S")),
                                         float(tol), int(max_iter),
                                         ctypes.c_void_p(_dev_ptr(out, self.shape, "out"))), "mbs_solve_async")
        self._keep[slot] = (S, out)

    def poll(self, slot: int):
        """None while the slot is running (``self.progress[slot]`` then holds the iterations and
        relative residual of its last completed launch), else its result dict (raises on a solve
        error)."""
        res = Result()
        st = self._lib.mbs_poll(self._h, int(slot), ctypes.byref(res))
        if st == MBS_EBUSY:
            self.progress[int(slot)] = (res.iterations, res.rel_residual)
            return None
        self._keep.pop(slot, None)
        _check(st, "mbs_poll")
        return res.as_dict()

    def residual(self, slot: int, field: Optional[torch.Tensor] = None) -> float:
        out = ctypes.c_double(0.0)
        ptr = ctypes.c_void_p(_dev_ptr(field, self.shape, "field")) if field is not None else ctypes.c_void_p(0)
        _check(self._lib.mbs_residual(self._h, int(slot), ptr, ctypes.byref(out)), "mbs_residual")
        return float(out.value)

    def history(self, slot: int, max_n: int = 1 << 16):
        buf = (ctypes.c_double * max_n)()
        n = ctypes.c_int32(0)
        _check(self._lib.mbs_residual_history(self._h, int(slot), buf, int(max_n), ctypes.byref(n)),
               "mbs_residual_history")
        return [buf[i] for i in range(n.value)]

    def timing(self, reset: bool = False) -> dict:
        nk = len(KERNEL_KINDS)
        ms = (ctypes.c_double * nk)()
        cnt = (ctypes.c_int64 * nk)()
        _check(self._lib.mbs_timing_read(self._h, ms, cnt, nk, int(reset)), "mbs_timing_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}
