"""Thin Python binding of libfosb.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only converts
torch tensors / numpy arrays to the C ABI's pointers and sizes, allocates
output tensors with torch on the context's device, and turns non-OK
statuses into FosbError.  The names mirror include/fosb.h.
"""

from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfosb.so")

FP64, MIXED = 0, 1
GAUSSIAN, MATERN32, CONSTANT, NORMAL_DOT = 0, 1, 2, 3
RADIAL, NORMAL = 0, 1
STATUS = {0: "OK", 1: "E_INVALID", 2: "E_SINGULAR", 3: "E_NOCONV", 4: "E_WORKSPACE", 5: "E_OOM",
          6: "E_DEVICE", 7: "E_UNSUPPORTED"}
COV_KINDS = {"gaussian": GAUSSIAN, "matern32": MATERN32, "constant": CONSTANT, "normal_dot": NORMAL_DOT}
FIELDS = {"radial": RADIAL, "normal": NORMAL}
FORM_EFIE, FORM_PMCHWT = 0, 1
FACTOR_LU, FACTOR_SYM = 0, 1
SD_STREAMED = 16


class FosbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Opts(C.Structure):
    _fields_ = [("n_gauss_singular", C.c_int32), ("ir_max_sweeps", C.c_int32), ("ir_tol", C.c_double),
                ("certify", C.c_int32), ("lu_pivoting", C.c_int32)]


class Cov(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("sigma", C.c_double), ("ell", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("ir_sweeps", C.c_int32), ("n_solves", C.c_int32), ("ir_rel_correction", C.c_double),
                ("backward_error", C.c_double), ("kappa1", C.c_double), ("growth", C.c_double)]


class BatchShape(C.Structure):
    _fields_ = [("meshes", C.POINTER(C.c_void_p)), ("n_levels", C.c_int32), ("L0", C.c_int32), ("L", C.c_int32),
                ("field", C.c_int32), ("k", C.c_double), ("dirs", C.c_void_p), ("pols", C.c_void_p),
                ("n_dirs", C.c_int64), ("cov", Cov), ("var", C.c_void_p)]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_D = C.c_double
_SIGS = {
    "fosb_last_error": (C.c_char_p, []),
    "fosb_opts_default": (C.c_int, [C.POINTER(Opts)]),
    "fosb_context_create": (C.c_int, [_I32, _P, C.POINTER(_P)]),
    "fosb_context_destroy": (C.c_int, [_P]),
    "fosb_context_synchronize": (C.c_int, [_P]),
    "fosb_context_memory": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "fosb_context_trim": (C.c_int, [_P]),
    "fosb_mesh_validate": (C.c_int, [_P, _I64, _P, _I64, C.POINTER(_I64)]),
    "fosb_mesh_create": (C.c_int, [_P, _P, _I64, _P, _I64, C.POINTER(_P)]),
    "fosb_mesh_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "fosb_mesh_destroy": (C.c_int, [_P]),
    "fosb_assemble": (C.c_int, [_P, _P, _D, C.POINTER(Opts), _P, _I64]),
    "fosb_level_create": (C.c_int, [_P, _P, _D, _I32, _P, _I64, _P, _I64, _P, _P, _I64, _I32, C.POINTER(Opts),
                                    C.POINTER(_P)]),
    "fosb_assemble_pmchwt": (C.c_int, [_P, _P, _D, _D, _D, C.POINTER(Opts), _P, _I64]),
    "fosb_level_create_pmchwt": (C.c_int, [_P, _P, _D, _D, _D, _I32, _P, _I64, _P, _I64, _P, _P, _I64, _I32,
                                           C.POINTER(Opts), C.POINTER(_P)]),
    "fosb_level_formulation": (C.c_int, [_P, C.POINTER(_I32), C.POINTER(_D), C.POINTER(_D)]),
    "fosb_level_factorization": (C.c_int, [_P, C.POINTER(_I32)]),
    "fosb_level_sd_weights": (C.c_int, [_P, _P, _I64, _P, _I64]),
    "fosb_level_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I64)]),
    "fosb_level_workspace_size": (C.c_int, [_P, _I32, _I64, _I64, C.POINTER(_I64), C.POINTER(_I64)]),
    "fosb_level_certificate": (C.c_int, [_P, C.POINTER(_D), C.POINTER(_D)]),
    "fosb_level_solve": (C.c_int, [_P, _P, _P, _I64, _I64, C.POINTER(Stats)]),
    "fosb_level_solve_adjoint": (C.c_int, [_P, _P, _P, _I64, _I64, C.POINTER(Stats)]),
    "fosb_level_first_moment": (C.c_int, [_P, _P, _I64, _P]),
    "fosb_level_destroy": (C.c_int, [_P]),
    "fosb_rhs_correlation": (C.c_int, [_P, _P, _P, C.POINTER(Cov), _I64, _P, _I64]),
    "fosb_two_sided_solve": (C.c_int, [_P, _P, _P, _P, _I64, C.POINTER(Stats)]),
    "fosb_ct_pairs": (C.c_int, [_I32, _I32, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32),
                                C.POINTER(_I32)]),
    "fosb_correlation": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(Cov), _I64, C.POINTER(_P),
                                   C.POINTER(_I64), C.POINTER(Stats)]),
    "fosb_far_field_matrix": (C.c_int, [_P, _P, _P, _I64, _P]),
    "fosb_far_field_moments": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(_P), C.POINTER(_I64), _P,
                                         _I64, _I64, _P, _P, _P]),
    "fosb_far_field_variance_adjoint": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(Cov), _P, _I64,
                                                  _I64, _P, _P, C.POINTER(Stats)]),
    "fosb_lowrank_create": (C.c_int, [_P, C.POINTER(_P), _I32, C.POINTER(Cov), _I32, _D, C.POINTER(_P)]),
    "fosb_lowrank_info": (C.c_int, [_P, C.POINTER(_I32), C.POINTER(_D), C.POINTER(_I64)]),
    "fosb_lowrank_factor": (C.c_int, [_P, _P, _I32, _I64, _P, _I64, C.POINTER(Stats)]),
    "fosb_far_field_moments_lowrank": (C.c_int, [_P, _P, _I32, _I32, _P, _I64, _I64, _P, C.POINTER(Stats)]),
    "fosb_lowrank_destroy": (C.c_int, [_P]),
    "fosb_near_field_matrix": (C.c_int, [_P, _P, _P, _I64, _P]),
    "fosb_near_field_moments": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(_P), C.POINTER(_I64), _P,
                                          _I64, _I64, _P, _P]),
    "fosb_far_field_moments_noalloc": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(_P), C.POINTER(_I64),
                                                 _P, _I64, _I64, _P, _P]),
    "fosb_far_field_moments_backward": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, C.POINTER(Cov), _P, _I64,
                                                  _I64, _P, _P, C.POINTER(Stats)]),
    "fosb_second_moment": (C.c_int, [_P, C.POINTER(_P), _I32, _I32, _I32, _D, _I32, C.POINTER(_P), C.POINTER(_I64),
                                     C.POINTER(_P), C.POINTER(_I64), _P, _P, _I64, _I32, C.POINTER(Cov), _I64, _P,
                                     _I64, C.POINTER(_P), C.POINTER(_I64), _P, C.POINTER(Opts), C.POINTER(_P),
                                     C.POINTER(Stats)]),
    "fosb_second_moment_batch": (C.c_int, [_P, C.POINTER(BatchShape), _I64, _I32, _P, _I64, C.POINTER(Opts), _I32,
                                           C.POINTER(Stats)]),
    "fosb_autotune": (C.c_int, [_P, _I32, C.POINTER(_I32)]),
    "fosb_autotune_table": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I32), _I64, C.POINTER(_I64)]),
    "fosb_autotune_load": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I32), _I64]),
    "fosb_profile_enable": (C.c_int, [_P, _I32]),
    "fosb_profile_read": (C.c_int, [_P, _I32, C.POINTER(_I64), C.POINTER(_D), C.POINTER(_D), C.POINTER(_D)]),
}

KERNEL_CLASSES = {"gemm_f64": 0, "gemm_f32": 1, "assemble": 2, "panel": 3, "trsm_leaf": 4, "rhs": 5, "gemv": 6, "splitk_sum": 7}

_lib = None


def lib() -> C.CDLL:
    """Load libfosb.so (built in-tree).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_01457_amd.build` "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise FosbError(status, lib().fosb_last_error().decode())


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _dev(t, dtype=None):
    """Device pointer of a contiguous torch CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def opts_default(**kw) -> Opts:
    o = Opts()
    _check(lib().fosb_opts_default(C.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def level_workspace_size(mesh: "Mesh", precision: int, n_dirs: int = 1, nrhs: int = 0) -> tuple[int, int]:
    """fosb_level_workspace_size: (bytes a level keeps, largest work buffer bytes)."""
    a, b = _I64(), _I64()
    _check(lib().fosb_level_workspace_size(mesh.h, precision, n_dirs, nrhs, C.byref(a), C.byref(b)))
    return a.value, b.value


def mesh_validate(V, F) -> int:
    """Host-only validation; returns the number of RWG functions (edges)."""
    V = _host_f64(V)
    F = _host_i32(F)
    ne = _I64()
    _check(lib().fosb_mesh_validate(V.ctypes.data_as(_P), V.shape[0], F.ctypes.data_as(_P), F.shape[0], C.byref(ne)))
    return ne.value


def ct_pairs(L0: int, L: int) -> list[tuple[int, int, int, int]]:
    n = L - L0 + 1
    a, b, s, m = ((_I32 * n)() for _ in range(4))
    cnt = _I32()
    _check(lib().fosb_ct_pairs(L0, L, a, b, s, m, C.byref(cnt)))
    return [(a[i], b[i], s[i], m[i]) for i in range(cnt.value)]


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = _P()
        _check(lib().fosb_context_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def synchronize(self):
        _check(lib().fosb_context_synchronize(self.h))

    def memory(self) -> dict:
        """fosb_context_memory: device allocations made, bytes cached for reuse, bytes in use."""
        a, c, u = _I64(), _I64(), _I64()
        _check(lib().fosb_context_memory(self.h, C.byref(a), C.byref(c), C.byref(u)))
        return {"n_device_allocs": a.value, "bytes_cached": c.value, "bytes_in_use": u.value}

    def trim(self):
        _check(lib().fosb_context_trim(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().fosb_context_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):   # bound now: `sys` may be gone at teardown
        if _finalizing():   # process teardown: the driver reclaims everything
            return
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx: "Context", mode: int = -1) -> int:
    """fosb_autotune: 0 off, 1 on, 2 on with a fresh table, -1 query.  Returns the
    number of tuned GEMM size buckets."""
    n = _I32()
    _check(lib().fosb_autotune(ctx.h, mode, C.byref(n)))
    return n.value


def autotune_table(ctx: "Context") -> dict:
    """fosb_autotune_table: the tuned table as {bucket key: tile variant}."""
    n = _I64()
    _check(lib().fosb_autotune_table(ctx.h, None, None, 0, C.byref(n)))
    cap = n.value
    keys = (_I64 * max(cap, 1))()
    var = (_I32 * max(cap, 1))()
    _check(lib().fosb_autotune_table(ctx.h, keys, var, cap, C.byref(n)))
    # the table may have grown between the two calls (tuning on another thread)
    return {int(keys[i]): int(var[i]) for i in range(min(n.value, cap))}


def autotune_load(ctx: "Context", table: dict) -> None:
    """fosb_autotune_load: add {bucket key: tile variant} entries to the table."""
    items = sorted((int(k), int(v)) for k, v in table.items())
    keys = (_I64 * max(len(items), 1))(*[k for k, _ in items])
    var = (_I32 * max(len(items), 1))(*[v for _, v in items])
    _check(lib().fosb_autotune_load(ctx.h, keys, var, len(items)))


def profile_enable(ctx: "Context", on: bool = True) -> None:
    _check(lib().fosb_profile_enable(ctx.h, 1 if on else 0))


def profile_read(ctx: "Context") -> dict:
    """{class: (launches, seconds, flops, bytes)} of the recorded launches."""
    out = {}
    for name, cls in KERNEL_CLASSES.items():
        n, s, f, b = _I64(), _D(), _D(), _D()
        _check(lib().fosb_profile_read(ctx.h, cls, C.byref(n), C.byref(s), C.byref(f), C.byref(b)))
        out[name] = (n.value, s.value, f.value, b.value)
    return out


class Mesh:
    def __init__(self, ctx: Context, V, F):
        self.ctx = ctx
        V = _host_f64(V)
        F = _host_i32(F)
        h = _P()
        _check(lib().fosb_mesh_create(ctx.h, V.ctypes.data_as(_P), V.shape[0], F.ctypes.data_as(_P), F.shape[0],
                                      C.byref(h)))
        self.h = h
        nt, ne, ntp = _I64(), _I64(), _I64()
        _check(lib().fosb_mesh_info(h, C.byref(nt), C.byref(ne), C.byref(ntp)))
        self.n_triangles, self.n_edges, self.n_touching = nt.value, ne.value, ntp.value

    def close(self):
        if getattr(self, "h", None):
            lib().fosb_mesh_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):   # bound now: `sys` may be gone at teardown
        if _finalizing():   # process teardown: the driver reclaims everything
            return
        try:
            self.close()
        except Exception:
            pass


def assemble(ctx: Context, mesh: Mesh, k: float, opts: Opts | None = None, Z=None):
    """fosb_assemble: returns the N x N complex128 EFIE matrix (torch, on device)."""
    import torch
    n = mesh.n_edges
    if Z is None:
        Z = torch.empty((n, n), dtype=torch.complex128, device=ctx.torch_device)
    _check(lib().fosb_assemble(ctx.h, mesh.h, float(k), C.byref(opts) if opts else None, _dev(Z, torch.complex128),
                               Z.stride(0)))
    return Z


def assemble_pmchwt(ctx: Context, mesh: Mesh, k0: float, eps_r: float, mu_r: float = 1.0,
                    opts: Opts | None = None, Z=None):
    """fosb_assemble_pmchwt: returns the 2N x 2N complex128 PMCHWT matrix (torch, on device)."""
    import torch
    n = 2 * mesh.n_edges
    if Z is None:
        Z = torch.empty((n, n), dtype=torch.complex128, device=ctx.torch_device)
    _check(lib().fosb_assemble_pmchwt(ctx.h, mesh.h, float(k0), float(eps_r), float(mu_r),
                                      C.byref(opts) if opts else None, _dev(Z, torch.complex128), Z.stride(0)))
    return Z


class Level:
    """fosb_level_create.  FP64: Z is factorised in place.  MIXED: Z is kept and
    a complex64 copy (allocated here unless given) receives the FP32 LU."""

    def __init__(self, ctx: Context, mesh: Mesh, k: float, Z, precision: int = FP64, dirs=((0.0, 0.0, 1.0),),
                 pols=((1.0, 0.0, 0.0),), field: str | int = "radial", opts: Opts | None = None, Zlow=None):
        import torch
        self.ctx, self.mesh, self.k, self.Z = ctx, mesh, float(k), Z
        self.precision = precision
        n = mesh.n_edges
        if precision == MIXED and Zlow is None:
            Zlow = torch.empty((n, n), dtype=torch.complex64, device=ctx.torch_device)
        self.Zlow = Zlow
        d = _host_f64(dirs).reshape(-1, 3)
        p = _host_f64(pols).reshape(-1, 3)
        fld = FIELDS[field] if isinstance(field, str) else int(field)
        h = _P()
        _check(lib().fosb_level_create(ctx.h, mesh.h, self.k, precision,
                                       _dev(Z, torch.complex128) if Z is not None else None,
                                       Z.stride(0) if Z is not None else 0,
                                       _dev(Zlow, torch.complex64) if Zlow is not None else None,
                                       Zlow.stride(0) if Zlow is not None else 0, d.ctypes.data_as(_P),
                                       p.ctypes.data_as(_P), d.shape[0], fld, C.byref(opts) if opts else None,
                                       C.byref(h)))
        self.h = h
        self.n = n
        self.n_dirs = d.shape[0]

    @classmethod
    def pmchwt(cls, ctx: "Context", mesh: "Mesh", k0: float, eps_r: float, mu_r: float, Z, precision: int = FP64,
               dirs=((0.0, 0.0, 1.0),), pols=((1.0, 0.0, 0.0),), opts: Opts | None = None, Zlow=None,
               field: str | int | None = None, streamed: bool = False):
        """fosb_level_create_pmchwt: a dielectric level on the 2N x 2N matrix Z
        of assemble_pmchwt (factorised in place for FP64, kept for MIXED);
        field ("radial" / "normal") also builds its shape-derivative weights,
        or, with streamed, recomputes them by source bands where the low-rank
        route needs them."""
        import torch
        self = cls.__new__(cls)
        self.ctx, self.mesh, self.k, self.Z = ctx, mesh, float(k0), Z
        self.precision = precision
        n = 2 * mesh.n_edges
        if precision == MIXED and Zlow is None:
            Zlow = torch.empty((n, n), dtype=torch.complex64, device=ctx.torch_device)
        self.Zlow = Zlow
        d = _host_f64(dirs).reshape(-1, 3)
        p = _host_f64(pols).reshape(-1, 3)
        h = _P()
        _check(lib().fosb_level_create_pmchwt(ctx.h, mesh.h, self.k, float(eps_r), float(mu_r), precision,
                                              _dev(Z, torch.complex128), Z.stride(0),
                                              _dev(Zlow, torch.complex64) if Zlow is not None else None,
                                              Zlow.stride(0) if Zlow is not None else 0, d.ctypes.data_as(_P),
                                              p.ctypes.data_as(_P), d.shape[0],
                                              -1 if field is None else (FIELDS[field] if isinstance(field, str)
                                                                        else int(field)) | (SD_STREAMED if streamed
                                                                                            else 0),
                                              C.byref(opts) if opts else None, C.byref(h)))
        self.h, self.n, self.n_dirs = h, n, d.shape[0]
        return self

    def sd_weights(self, dir: int = 0):
        """fosb_level_sd_weights: the dielectric shape-derivative weights (2N x 6 nt)."""
        import torch
        W = torch.empty((self.n, 6 * self.mesh.n_triangles), dtype=torch.complex128, device=self.ctx.torch_device)
        _check(lib().fosb_level_sd_weights(self.ctx.h, self.h, dir, _dev(W), W.stride(0)))
        return W

    def formulation(self) -> tuple[int, float, float]:
        """fosb_level_formulation: (FORM_EFIE or FORM_PMCHWT, eps_r, mu_r)."""
        f, e, m = _I32(), _D(), _D()
        _check(lib().fosb_level_formulation(self.h, C.byref(f), C.byref(e), C.byref(m)))
        return f.value, e.value, m.value

    def factorization(self) -> int:
        """fosb_level_factorization: FACTOR_LU or FACTOR_SYM."""
        k = _I32()
        _check(lib().fosb_level_factorization(self.h, C.byref(k)))
        return k.value

    def solve(self, B, stats: Stats | None = None):
        import torch
        st = stats if stats is not None else Stats()
        B2 = B if B.dim() == 2 else B.view(-1, 1)
        _check(lib().fosb_level_solve(self.ctx.h, self.h, _dev(B2, torch.complex128), B2.stride(0), B2.shape[1],
                                      C.byref(st)))
        return B

    @classmethod
    def _adopt(cls, ctx: "Context", mesh: "Mesh", k: float, h, precision: int, Z, Zlow, n_dirs: int):
        """Wrap a handle created by the library (fosb_second_moment)."""
        self = cls.__new__(cls)
        self.ctx, self.mesh, self.k, self.Z, self.Zlow = ctx, mesh, float(k), Z, Zlow
        self.precision, self.h, self.n, self.n_dirs = precision, h, mesh.n_edges, n_dirs
        return self

    def solve_adjoint(self, B, stats: Stats | None = None):
        """B <- Z^{-H} B in place."""
        import torch
        st = stats if stats is not None else Stats()
        B2 = B if B.dim() == 2 else B.view(-1, 1)
        _check(lib().fosb_level_solve_adjoint(self.ctx.h, self.h, _dev(B2, torch.complex128), B2.stride(0),
                                              B2.shape[1], C.byref(st)))
        return B

    def certificate(self) -> tuple[float, float]:
        """fosb_level_certificate: (1-norm condition estimate, growth factor); 0 without opts.certify."""
        k, g = _D(), _D()
        _check(lib().fosb_level_certificate(self.h, C.byref(k), C.byref(g)))
        return k.value, g.value

    def first_moment(self, dir: int = 0):
        import torch
        u = torch.empty(self.n, dtype=torch.complex128, device=self.ctx.torch_device)
        _check(lib().fosb_level_first_moment(self.ctx.h, self.h, dir, _dev(u)))
        return u

    def close(self):
        if getattr(self, "h", None):
            lib().fosb_level_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):   # bound now: `sys` may be gone at teardown
        if _finalizing():   # process teardown: the driver reclaims everything
            return
        try:
            self.close()
        except Exception:
            pass


def make_cov(kind: str | int, sigma: float, ell: float = 1.0) -> Cov:
    c = Cov()
    c.kind = COV_KINDS[kind] if isinstance(kind, str) else int(kind)
    c.sigma = float(sigma)
    c.ell = float(ell)
    return c


def rhs_correlation(ctx: Context, l1: Level, l2: Level, cov: Cov, dir: int = 0, C_out=None):
    import torch
    if C_out is None:
        C_out = torch.empty((l1.n, l2.n), dtype=torch.complex128, device=ctx.torch_device)
    _check(lib().fosb_rhs_correlation(ctx.h, l1.h, l2.h, C.byref(cov) if cov is not None else None, dir,
                                      _dev(C_out, torch.complex128), C_out.stride(0)))
    return C_out


def two_sided_solve(ctx: Context, l1: Level, l2: Level, C_io, stats: Stats | None = None):
    import torch
    st = stats if stats is not None else Stats()
    _check(lib().fosb_two_sided_solve(ctx.h, l1.h, l2.h, _dev(C_io, torch.complex128), C_io.stride(0), C.byref(st)))
    return C_io


def correlation(ctx: Context, levels: list[Level], L0: int, L: int, cov: Cov, dir: int = 0, blocks=None,
                stats: Stats | None = None):
    """All Sigma blocks of the Hermitian-reduced CT index set, in ct_pairs order."""
    import torch
    pairs = ct_pairs(L0, L)
    if blocks is None:
        blocks = [torch.empty((levels[a - L0].n, levels[b - L0].n), dtype=torch.complex128, device=ctx.torch_device)
                  for a, b, _, _ in pairs]
    st = stats if stats is not None else Stats()
    lv = (_P * len(levels))(*[l.h for l in levels])
    bp = (_P * len(blocks))(*[_dev(b, torch.complex128) for b in blocks])
    ld = (_I64 * len(blocks))(*[b.stride(0) for b in blocks])
    _check(lib().fosb_correlation(ctx.h, lv, len(levels), L0, L, C.byref(cov) if cov is not None else None, dir,
                                  bp, ld, C.byref(st)))
    return blocks


def far_field_matrix(ctx: Context, level: Level, xhat):
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    FF = torch.empty((3 * x.shape[0], level.n), dtype=torch.complex128, device=ctx.torch_device)
    _check(lib().fosb_far_field_matrix(ctx.h, level.h, x.ctypes.data_as(_P), x.shape[0], _dev(FF)))
    return FF


def far_field_moments(ctx: Context, levels: list[Level], L0: int, L: int, blocks, xhat, dir: int = 0,
                      with_mean: bool = False, with_cor: bool = False):
    """CT far-field variance (3, n_a) float64 on device, followed, when asked,
    by the angular correlation (3, n_a, n_a) complex128 and the finest level's
    mean far field (3, n_a)."""
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    n_a = x.shape[0]
    var = torch.empty(3 * n_a, dtype=torch.float64, device=ctx.torch_device)
    mean = torch.empty(3 * n_a, dtype=torch.complex128, device=ctx.torch_device) if with_mean else None
    cor = torch.empty((3, n_a, n_a), dtype=torch.complex128, device=ctx.torch_device) if with_cor else None
    lv = (_P * len(levels))(*[l.h for l in levels])
    bp = (_P * len(blocks))(*[_dev(b, torch.complex128) for b in blocks])
    ld = (_I64 * len(blocks))(*[b.stride(0) for b in blocks])
    _check(lib().fosb_far_field_moments(ctx.h, lv, len(levels), L0, L, bp, ld, x.ctypes.data_as(_P), n_a, dir,
                                        _dev(var, torch.float64), _dev(cor) if cor is not None else None,
                                        _dev(mean) if mean is not None else None))
    out = [var.view(3, n_a)]
    if with_cor:
        out.append(cor)
    if with_mean:
        out.append(mean.view(3, n_a))
    return out[0] if len(out) == 1 else tuple(out)


def far_field_variance_adjoint(ctx: Context, levels: list[Level], L0: int, L: int, cov: Cov, xhat, dir: int = 0,
                               with_mean: bool = False, stats: Stats | None = None):
    """fosb_far_field_variance_adjoint: the CT variance (3, n_a) without Sigma
    blocks [and the finest level's mean far field (3, n_a)]."""
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    n_a = x.shape[0]
    var = torch.empty(3 * n_a, dtype=torch.float64, device=ctx.torch_device)
    mean = torch.empty(3 * n_a, dtype=torch.complex128, device=ctx.torch_device) if with_mean else None
    st = stats if stats is not None else Stats()
    lv = (_P * len(levels))(*[l.h for l in levels])
    _check(lib().fosb_far_field_variance_adjoint(ctx.h, lv, len(levels), L0, L, C.byref(cov), x.ctypes.data_as(_P),
                                                 n_a, dir, _dev(var, torch.float64),
                                                 _dev(mean) if mean is not None else None, C.byref(st)))
    var = var.view(3, n_a)
    return (var, mean.view(3, n_a)) if with_mean else var


class LowRank:
    """fosb_lowrank_create: pivoted Cholesky factor of the covariance on the
    quadrature nodes of the ladder `levels` (coarse to fine)."""

    def __init__(self, ctx: Context, levels: list[Level], cov: Cov, max_rank: int, tol: float):
        self.ctx, self.levels = ctx, list(levels)
        lv = (_P * len(levels))(*[l.h for l in levels])
        h = _P()
        _check(lib().fosb_lowrank_create(ctx.h, lv, len(levels), C.byref(cov), int(max_rank), float(tol), C.byref(h)))
        self.h = h
        r, res = _I32(), _D()
        _check(lib().fosb_lowrank_info(h, C.byref(r), C.byref(res), None))
        self.rank, self.residual = r.value, res.value
        piv = (_I64 * max(self.rank, 1))()
        _check(lib().fosb_lowrank_info(h, None, None, piv))
        self.pivots = np.array([piv[i] for i in range(self.rank)], dtype=np.int64)

    def factor(self, level_index: int, dir: int = 0, stats: Stats | None = None):
        """Y = Z^{-1} Wgt L_l (N x rank, complex128 on the device)."""
        import torch
        n = self.levels[level_index].n
        Y = torch.empty((n, self.rank), dtype=torch.complex128, device=self.ctx.torch_device)
        st = stats if stats is not None else Stats()
        _check(lib().fosb_lowrank_factor(self.ctx.h, self.h, level_index, dir, _dev(Y, torch.complex128), Y.stride(0),
                                         C.byref(st)))
        return Y

    def far_field_moments(self, L0: int, L: int, xhat, dir: int = 0, stats: Stats | None = None):
        import torch
        x = _host_f64(xhat).reshape(-1, 3)
        var = torch.empty(3 * x.shape[0], dtype=torch.float64, device=self.ctx.torch_device)
        st = stats if stats is not None else Stats()
        _check(lib().fosb_far_field_moments_lowrank(self.ctx.h, self.h, L0, L, x.ctypes.data_as(_P), x.shape[0], dir,
                                                    _dev(var, torch.float64), C.byref(st)))
        return var.view(3, -1)

    def close(self):
        if getattr(self, "h", None):
            lib().fosb_lowrank_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):   # bound now: `sys` may be gone at teardown
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def near_field_matrix(ctx: Context, level: Level, points):
    import torch
    x = _host_f64(points).reshape(-1, 3)
    NF = torch.empty((3 * x.shape[0], level.n), dtype=torch.complex128, device=ctx.torch_device)
    _check(lib().fosb_near_field_matrix(ctx.h, level.h, x.ctypes.data_as(_P), x.shape[0], _dev(NF)))
    return NF


def near_field_moments(ctx: Context, levels: list[Level], L0: int, L: int, blocks, points, dir: int = 0):
    """CT variance of the field's shape derivative at field points (3, n_p)
    float64 and the finest level's scattered field there (3, n_p) complex128."""
    import torch
    x = _host_f64(points).reshape(-1, 3)
    n_p = x.shape[0]
    var = torch.empty(3 * n_p, dtype=torch.float64, device=ctx.torch_device)
    mean = torch.empty(3 * n_p, dtype=torch.complex128, device=ctx.torch_device)
    lv = (_P * len(levels))(*[l.h for l in levels])
    bp = (_P * len(blocks))(*[_dev(b, torch.complex128) for b in blocks])
    ld = (_I64 * len(blocks))(*[b.stride(0) for b in blocks])
    _check(lib().fosb_near_field_moments(ctx.h, lv, len(levels), L0, L, bp, ld, x.ctypes.data_as(_P), n_p, dir,
                                         _dev(var, torch.float64), _dev(mean)))
    return var.view(3, n_p), mean.view(3, n_p)


def far_field_moments_noalloc(ctx: Context, levels: list[Level], L0: int, L: int, blocks, xhat, var, dir: int = 0,
                              mean=None):
    """fosb_far_field_moments_noalloc into caller tensors: var (3 n_a) float64
    and optionally mean (3 n_a) complex128, both on the device."""
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    lv = (_P * len(levels))(*[l.h for l in levels])
    bp = (_P * len(blocks))(*[_dev(b, torch.complex128) for b in blocks])
    ld = (_I64 * len(blocks))(*[b.stride(0) for b in blocks])
    _check(lib().fosb_far_field_moments_noalloc(ctx.h, lv, len(levels), L0, L, bp, ld, x.ctypes.data_as(_P),
                                                x.shape[0], dir, _dev(var, torch.float64),
                                                _dev(mean, torch.complex128) if mean is not None else None))
    return var


def far_field_moments_backward(ctx: Context, levels: list[Level], L0: int, L: int, cov: Cov, xhat, dvar,
                               dir: int = 0, stats: Stats | None = None):
    """Adjoint of the CT variance in the covariance parameters: for S = sum(dvar * var)
    returns a device float64 tensor (dS/dsigma, dS/dell, S)."""
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    n_a = x.shape[0]
    g = dvar.reshape(3 * n_a)
    if not g.is_contiguous():
        g = g.contiguous()
    out = torch.empty(3, dtype=torch.float64, device=ctx.torch_device)
    st = stats if stats is not None else Stats()
    lv = (_P * len(levels))(*[l.h for l in levels])
    _check(lib().fosb_far_field_moments_backward(ctx.h, lv, len(levels), L0, L, C.byref(cov), x.ctypes.data_as(_P),
                                                 n_a, dir, _dev(g, torch.float64), _dev(out, torch.float64),
                                                 C.byref(st)))
    return out


def _variance_function():
    import torch

    class RcsVariance(torch.autograd.Function):
        """var(sigma, ell) through fosb_correlation + fosb_far_field_moments; the
        backward pass is fosb_far_field_moments_backward."""

        @staticmethod
        def forward(fctx, sigma, ell, ctx, levels, L0, L, kind, xhat, dir):
            cov = make_cov(kind, float(sigma), float(ell))
            blocks = correlation(ctx, levels, L0, L, cov, dir)
            var = far_field_moments(ctx, levels, L0, L, blocks, xhat, dir)
            del blocks
            fctx.args = (ctx, levels, L0, L, cov, xhat, dir)
            fctx.devices = (sigma.device, ell.device)
            return var

        @staticmethod
        def backward(fctx, gvar):
            ctx, levels, L0, L, cov, xhat, dir = fctx.args
            g = gvar.to(torch.float64).contiguous()
            out = far_field_moments_backward(ctx, levels, L0, L, cov, xhat, g, dir)
            return (out[0].to(fctx.devices[0]), out[1].to(fctx.devices[1]), None, None, None, None, None, None,
                    None)

    return RcsVariance


_RCS_VARIANCE = None


def rcs_variance(ctx: Context, levels: list[Level], L0: int, L: int, kind: str, sigma, ell, xhat, dir: int = 0):
    """Differentiable CT far-field variance (3, n_a) as a function of the covariance
    amplitude sigma and correlation length ell (0-d float64 tensors)."""
    global _RCS_VARIANCE
    if _RCS_VARIANCE is None:
        _RCS_VARIANCE = _variance_function()
    return _RCS_VARIANCE.apply(sigma, ell, ctx, levels, L0, L, kind, xhat, dir)


def second_moment(ctx: Context, meshes: list[Mesh], L0: int, L: int, k: float, precision: int, cov: Cov, xhat,
                  dirs=((0.0, 0.0, 1.0),), pols=((1.0, 0.0, 0.0),), field: str | int = "radial", dir: int = 0,
                  Z=None, Zlow=None, blocks=None, opts: Opts | None = None, keep_levels: bool = False,
                  stats: Stats | None = None):
    """fosb_second_moment: the whole hot path over the ladder meshes (levels
    L0..L, coarse to fine) with the library's two-stream schedule.  Returns
    (var (3, n_a), blocks, levels or None); dir = -1 solves every incidence
    together (blocks N1 x n_dirs*N2, var (n_dirs, 3, n_a))."""
    import torch
    n = len(meshes)
    dev = ctx.torch_device
    if Z is None:
        Z = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex128, device=dev) for m in meshes]
    if precision == MIXED and Zlow is None:
        Zlow = [torch.empty((m.n_edges, m.n_edges), dtype=torch.complex64, device=dev) for m in meshes]
    pairs = ct_pairs(L0, L)
    x = _host_f64(xhat).reshape(-1, 3)
    d = _host_f64(dirs).reshape(-1, 3)
    p = _host_f64(pols).reshape(-1, 3)
    nd = d.shape[0] if dir < 0 else 1
    if blocks is None:
        blocks = [torch.empty((meshes[a - L0].n_edges, nd * meshes[b - L0].n_edges), dtype=torch.complex128,
                              device=dev) for a, b, _, _ in pairs]
    var = torch.empty(nd * 3 * x.shape[0], dtype=torch.float64, device=dev)
    st = stats if stats is not None else Stats()
    ms = (_P * n)(*[m.h for m in meshes])
    zp = (_P * n)(*[_dev(z, torch.complex128) if z is not None else None for z in Z])
    zl = (_I64 * n)(*[z.stride(0) if z is not None else 0 for z in Z])
    if precision == MIXED:
        lp = (_P * n)(*[_dev(z, torch.complex64) for z in Zlow])
        ll = (_I64 * n)(*[z.stride(0) for z in Zlow])
    else:
        lp, ll = None, None
    bp = (_P * len(blocks))(*[_dev(b, torch.complex128) for b in blocks])
    bl = (_I64 * len(blocks))(*[b.stride(0) for b in blocks])
    out = (_P * n)() if keep_levels else None
    fld = FIELDS[field] if isinstance(field, str) else int(field)
    _check(lib().fosb_second_moment(ctx.h, ms, n, L0, L, float(k), precision, zp, zl, lp, ll, d.ctypes.data_as(_P),
                                    p.ctypes.data_as(_P), d.shape[0], fld, C.byref(cov), dir, x.ctypes.data_as(_P),
                                    x.shape[0], bp, bl, _dev(var, torch.float64), C.byref(opts) if opts else None,
                                    out, C.byref(st)))
    levels = None
    if keep_levels:
        levels = [Level._adopt(ctx, meshes[i], k, _P(out[i]), precision, Z[i],
                               Zlow[i] if precision == MIXED else None, d.shape[0]) for i in range(n)]
    return (var.view(3, -1) if dir >= 0 else var.view(nd, 3, -1)), blocks, levels


def second_moment_batch(ctx: Context, shapes, precision: int, xhat, opts: Opts | None = None, n_workers: int = 4,
                        stats: Stats | None = None):
    """fosb_second_moment_batch.  shapes: list of dicts with keys meshes (list of
    Mesh, coarse to fine), L0, L, k, dirs, pols, cov (Cov) and optionally field.
    Returns one device tensor (n_dirs, 3, n_a) per shape."""
    import torch
    x = _host_f64(xhat).reshape(-1, 3)
    arr = (BatchShape * len(shapes))()
    keep = []
    outs = []
    for i, sh in enumerate(shapes):
        d = _host_f64(sh["dirs"]).reshape(-1, 3)
        p = _host_f64(sh["pols"]).reshape(-1, 3)
        ms = (_P * len(sh["meshes"]))(*[m.h for m in sh["meshes"]])
        var = torch.empty((d.shape[0], 3, x.shape[0]), dtype=torch.float64, device=ctx.torch_device)
        fld = sh.get("field", "radial")
        b = arr[i]
        b.meshes = C.cast(ms, C.POINTER(C.c_void_p))
        b.n_levels, b.L0, b.L = len(sh["meshes"]), sh["L0"], sh["L"]
        b.field = FIELDS[fld] if isinstance(fld, str) else int(fld)
        b.k = float(sh["k"])
        b.dirs, b.pols, b.n_dirs = d.ctypes.data_as(_P), p.ctypes.data_as(_P), d.shape[0]
        b.cov = sh["cov"]
        b.var = _dev(var, torch.float64)
        keep += [d, p, ms]
        outs.append(var)
    st = stats if stats is not None else Stats()
    _check(lib().fosb_second_moment_batch(ctx.h, arr, len(shapes), precision, x.ctypes.data_as(_P), x.shape[0],
                                          C.byref(opts) if opts else None, n_workers, C.byref(st)))
    del keep
    return outs


@dataclass
class PipelineResult:
    var: object            # (3, n_a) float64 device tensor
    blocks: list           # Sigma blocks (device)
    levels: list           # Level handles (keep alive with the blocks)
    meshes: list
    stats: Stats


def run_pipeline(ctx: Context, meshes_VF, k: float, L0: int, L: int, cov: Cov, xhat, precision: int = FP64,
                 dirs=((0.0, 0.0, 1.0),), pols=((1.0, 0.0, 0.0),), field="radial", opts: Opts | None = None,
                 dir: int = 0) -> PipelineResult:
    """One pass of the hot path: assemble every level (L0..L), factorise and solve
    the first moments, then all CT level-pair solves and the far-field variance.
    meshes_VF: list of (V, F) for levels L0..L."""
    meshes = [Mesh(ctx, V, F) for V, F in meshes_VF]
    levels = []
    for m in meshes:
        Z = assemble(ctx, m, k, opts)
        levels.append(Level(ctx, m, k, Z, precision, dirs, pols, field, opts))
    st = Stats()
    blocks = correlation(ctx, levels, L0, L, cov, dir, stats=st)
    var = far_field_moments(ctx, levels, L0, L, blocks, xhat, dir)
    return PipelineResult(var, blocks, levels, meshes, st)
