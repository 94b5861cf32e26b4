"""Python binding of libmg.so, the MI355X geometric multigrid library.

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Functions carry the C names of ``include/mg.h``; arrays are torch
tensors on the HIP device (their ``data_ptr()`` is passed), the stream is
torch's current stream unless one is given.  Importing this package never
touches a GPU; the first call that needs ``libmg.so`` loads it and raises if
it has not been built (``python -m paper_1406_5369_amd.build``).
"""

from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import re
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mg.h")

# status codes (enum mg_status)
MG_OK, MG_ENOTCONV, MG_EINVAL, MG_ENOTSUP, MG_ENOMEM, MG_EDEVICE, MG_EDIVERGED, MG_EBUSY = 0, 1, -1, -2, -3, -4, -5, -6
OP_LAPLACE, OP_CONST_STENCIL, OP_VARCOEF_NODAL = 0, 1, 2
BC_DIRICHLET_ZERO, BC_NEUMANN_CC = 0, 1
SMOOTH_RBGS, SMOOTH_JACOBI, SMOOTH_RBGS_SYM = 0, 1, 2
CYCLE_V, CYCLE_W, CYCLE_F = 0, 1, 2
PREC_FP64, PREC_FP32_IR, PREC_FP16_IR = 0, 1, 2


class MGError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_int),
        ("op", C.c_int),
        ("k", C.c_void_p),
        ("bc", C.c_int),
        ("smoother", C.c_int),
        ("omega", C.c_double),
        ("nu1", C.c_int),
        ("nu2", C.c_int),
        ("precision", C.c_int),
        ("cycle", C.c_int),
        ("coarse_n", C.c_int),
        ("cg_iters", C.c_int),
        ("stencil", C.c_void_p),
        ("h", C.c_double),
    ]


class _CDiffParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_int),
        ("tau", C.c_double),
        ("theta", C.c_double),
        ("k", C.c_double),
        ("smoother", C.c_int),
        ("omega", C.c_double),
        ("nu1", C.c_int),
        ("nu2", C.c_int),
    ]


class _ServerParams(C.Structure):
    _fields_ = [
        ("hbm_budget_bytes", C.c_size_t),
        ("max_slots", C.c_int),
        ("max_n2d", C.c_int),
        ("max_n3d", C.c_int),
        ("smoother", C.c_int),
        ("omega", C.c_double),
        ("nu1", C.c_int),
        ("nu2", C.c_int),
        ("tol", C.c_double),
        ("max_cycles", C.c_int),
    ]


_lib = None


def lib():
    """Load libmg.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1406_5369_amd.build`")
        L = C.CDLL(LIB_PATH)
        i, d, p, sz = C.c_int, C.c_double, C.c_void_p, C.c_size_t
        sig = {
            "mg_setup": (i, [C.POINTER(_Params), p, C.POINTER(p)]),
            "mg_destroy": (None, [p]),
            "mg_vcycle": (i, [p, p, p]),
            "mg_solve": (i, [p, p, p, d, i, C.POINTER(i), p]),
            "mg_residual_norm": (i, [p, p, p, C.POINTER(d)]),
            "mg_num_levels": (i, [p]),
            "mg_tile_config": (i, [p, i, i, C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(i),
                                   C.POINTER(i)]),
            "mg_strerror": (C.c_char_p, [i]),
            "mg_level_smooth": (i, [i, i, i, i, d, p, p, p, p, p, i, i, i, i, i, i, p]),
            "mg_level_residual_restrict": (i, [i, i, i, p, p, p, p, i, i, p]),
            "mg_level_prolong_correct": (i, [i, i, i, p, p, p]),
            "mg_level_coarsest": (i, [i, i, p, p, p, p]),
            "mg_level_smooth_restrict": (i, [i, i, i, p, p, p, p, i, i, p]),
            "mg_level_smooth2_zero": (i, [i, i, i, p, p, i, i, i, p]),
            "mg_level_smooth2_correct": (i, [i, i, i, i, p, p, p, p, i, i, p]),
            "mg_level_coarsest_cg": (i, [i, i, i, p, p, p, i, p]),
            "mg_cdiff_setup": (i, [C.POINTER(_CDiffParams), p, C.POINTER(p)]),
            "mg_cdiff_fas": (i, [p, p, p]),
            "mg_cdiff_apply": (i, [p, p, p]),
            "mg_cdiff_run": (i, [p, p, i, d, i, p, p]),
            "mg_level_st_smooth": (i, [i, i, p, i, d, p, p, p, p]),
            "mg_level_st_residual_restrict": (i, [i, i, p, p, p, p, p]),
            "mg_level_st_coarsest": (i, [i, p, p, p, p]),
            "mg_level_cc_smooth": (i, [i, i, i, d, p, p, p, p]),
            "mg_level_cc_residual_restrict": (i, [i, i, p, p, p, p]),
            "mg_level_cc_prolong_correct": (i, [i, i, p, p, p]),
            "mg_level_cc_remove_mean": (i, [i, i, p, C.POINTER(d), p]),
            "mg_level_ir_update": (i, [i, i, p, p, p, p, p, p, C.POINTER(d), i, i, i, i, i, p]),
            "mg_level_ir_update_noalloc": (i, [i, i, p, p, p, p, p, p, C.POINTER(d), i, i, i, i, i, p]),
            "mg_level_ir_update_f16": (i, [i, i, p, p, d, d, p, p, p, C.POINTER(d), C.POINTER(d), i, i, i, i, p]),
            "mg_prof_enable": (i, [p, i]),
            "mg_prof_read": (i, [p, C.POINTER(i), C.POINTER(d)]),
            "mg_prof_read_kernel": (i, [p, i, C.POINTER(i), C.POINTER(d)]),
            "mg_copy_kernel": (i, [p, p, sz, p]),
            "mg_batch_setup": (i, [i, p, p, C.POINTER(p)]),
            "mg_batch_solve": (i, [p, p, p, d, i, p, p]),
            "mg_server_create": (i, [C.POINTER(_ServerParams), p, C.POINTER(p)]),
            "mg_server_submit": (i, [p, i, i, p, C.POINTER(C.c_longlong)]),
            "mg_server_submit_device": (i, [p, i, i, p, p, C.POINTER(C.c_longlong)]),
            "mg_server_step": (i, [p, C.POINTER(i), C.POINTER(i)]),
            "mg_server_poll": (i, [p, p, i, C.POINTER(i)]),
            "mg_server_fetch": (i, [p, C.c_longlong, p, C.POINTER(i), C.POINTER(d), C.POINTER(d)]),
            "mg_server_info": (i, [p, C.POINTER(sz), C.POINTER(i), C.POINTER(i)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of every function declared in include/mg.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def strerror(code: int) -> str:
    try:
        return lib().mg_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def _check(code: int, where: str, ok=(MG_OK,)) -> int:
    if code not in ok:
        raise MGError(code, where)
    return code


def _stream(stream) -> Optional[int]:
    import torch

    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t, dtype=None, shape=None, name="array"):
    """Device pointer of a contiguous torch tensor on the HIP device (None -> NULL)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the HIP device")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


@dataclass
class Params:
    """Problem and solver parameters (struct mg_params).  Defaults are the paper's:
    V(2,2) cycles (Section 4), RBGS with omega = 1.0 (Section 2.3 Layer-3
    parameters) or Jacobi with omega = 0.8 (Table 2 caption)."""

    dim: int
    n: int
    op: int = OP_LAPLACE
    k: object = None  # torch float64 tensor of shape (n,)*dim for OP_VARCOEF_NODAL
    bc: int = BC_DIRICHLET_ZERO
    smoother: int = SMOOTH_RBGS
    omega: float = 0.0
    nu1: int = 2
    nu2: int = 2
    precision: int = PREC_FP64
    cycle: int = CYCLE_V
    coarse_n: int = 0  # 0 / 3: exact 3-node coarsest solve; larger: conjugate gradients there
    cg_iters: int = 0  # 0: 4 (coarse_n - 1)
    stencil: object = None  # OP_CONST_STENCIL: 2*dim + 1 coefficients, centre first, then -x, +x, -y, +y[, -z, +z]
    h: float = 0.0  # 0: the unit domain's spacing

    def __post_init__(self):
        if self.omega <= 0.0:
            self.omega = 0.8 if self.smoother == SMOOTH_JACOBI else 1.0

    @property
    def shape(self):
        return (self.n,) * self.dim

    def to_c(self) -> _Params:
        import torch

        kp = _dptr(self.k, torch.float64, self.shape, "k") if self.k is not None else None
        st = None
        if self.stencil is not None:
            vals = [float(x) for x in self.stencil]
            st = (C.c_double * len(vals))(*vals)
        cp = _Params(self.dim, self.n, self.op, kp, self.bc, self.smoother, self.omega, self.nu1, self.nu2,
                     self.precision, self.cycle, self.coarse_n, self.cg_iters,
                     C.cast(st, C.c_void_p) if st is not None else None, float(self.h))
        cp._stencil_buf = st  # keeps the host array alive while the structure is in use
        return cp


# Handles created through this module and not yet destroyed, in creation
# order.  They are destroyed explicitly (newest first, after the device has
# finished its work) when the interpreter exits, while the HIP runtime is
# still fully alive, instead of being left to object finalizers that may run
# during interpreter teardown.
_live: dict = {}


def _track(ctx: int) -> int:
    _live[ctx] = True
    return ctx


def mg_setup(params: Params, stream=None) -> int:
    """Create a context (returns the opaque handle as an int)."""
    cp = params.to_c()
    out = C.c_void_p()
    _check(lib().mg_setup(C.byref(cp), _stream(stream), C.byref(out)), "mg_setup")
    return _track(out.value)


def mg_destroy(ctx: int) -> None:
    if not ctx:
        return
    _live.pop(ctx, None)
    lib().mg_destroy(ctx)
    for key in [k for k in _server_shapes if k[0] == ctx]:
        del _server_shapes[key]


def shutdown() -> None:
    """Destroy every handle still alive (newest first) after the device has
    drained.  Registered with atexit; safe to call more than once."""
    if not _live or _lib is None:
        _live.clear()
        return
    try:
        import torch

        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for ctx in reversed(list(_live)):
        mg_destroy(ctx)


atexit.register(shutdown)


def mg_num_levels(ctx: int) -> int:
    return lib().mg_num_levels(ctx)


def mg_tile_config(ctx: int, level: int, family: int, with_order: bool = False):
    """(by, zchunk, prefetch, waves) used on a level by a kernel family (0 smooth, 1 restrict, 2 norm,
    3 smooth from a zero iterate, 4 smooth with the fused coarse-grid correction, 5 last pre-smoothing
    sweep fused with the restriction, 6 FP64 first pre-smoothing sweep that also sums the residual norm,
    all 0 when the norm is a pass of its own, 7 the first two pre-smoothing sweeps from a zero iterate in
    one launch, 8 the first two post-smoothing sweeps in one launch (2D), zchunk 0 when they run apart);
    with_order adds the block order (0 XCD bands, 1 linear)
    and the pairs flag (3D pass with two nodes per lane)."""
    by, zc, pd, wv, od, xp = (C.c_int(0) for _ in range(6))
    _check(lib().mg_tile_config(ctx, level, family, C.byref(by), C.byref(zc), C.byref(pd), C.byref(wv),
                                C.byref(od), C.byref(xp)), "mg_tile_config")
    if with_order:
        return by.value, zc.value, pd.value, wv.value, od.value, xp.value
    return by.value, zc.value, pd.value, wv.value


def mg_vcycle(ctx: int, u, f) -> None:
    import torch

    _check(lib().mg_vcycle(ctx, _dptr(u, torch.float64, name="u"), _dptr(f, torch.float64, name="f")), "mg_vcycle")


def mg_solve(ctx: int, u, f, tol: float = 1e-8, max_cycles: int = 50):
    """Returns (status, cycles, residual history as a list)."""
    import torch

    hist = (C.c_double * (max_cycles + 1))()
    cyc = C.c_int(0)
    st = lib().mg_solve(ctx, _dptr(u, torch.float64, name="u"), _dptr(f, torch.float64, name="f"), float(tol),
                        int(max_cycles), C.byref(cyc), hist)
    _check(st, "mg_solve", ok=(MG_OK, MG_ENOTCONV, MG_EDIVERGED))
    return st, cyc.value, list(hist[: cyc.value + 1])


def mg_residual_norm(ctx: int, u, f) -> float:
    import torch

    out = C.c_double(0.0)
    _check(lib().mg_residual_norm(ctx, _dptr(u, torch.float64, name="u"), _dptr(f, torch.float64, name="f"),
                                  C.byref(out)), "mg_residual_norm")
    return out.value


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    if t.dtype == torch.float16:
        return 2
    raise TypeError("arrays must be float64, float32 or float16")


def mg_level_smooth(u_in, f, u_out, smoother=SMOOTH_RBGS, omega=0.0, k=None, ec=None, zero_guess=False, by=0,
                    zchunk=0, prefetch=0, waves=0, order=0, stream=None) -> None:
    dim, n = f.dim(), f.shape[0]
    if omega <= 0.0:
        omega = 0.8 if smoother == SMOOTH_JACOBI else 1.0
    dt = f.dtype
    _check(lib().mg_level_smooth(dim, n, _dtype_code(f), smoother, float(omega), _dptr(k, dt, f.shape, "k"),
                                 _dptr(u_in, dt, f.shape, "u_in"), _dptr(f, dt, None, "f"),
                                 _dptr(u_out, dt, f.shape, "u_out"), _dptr(ec, dt, ((n - 1) // 2 + 1,) * dim, "ec"), int(zero_guess),
                                 by, zchunk, prefetch, waves, order, _stream(stream)), "mg_level_smooth")


def mg_level_residual_restrict(u, f, fc, k=None, by=0, zchunk=0, stream=None) -> None:
    dim, n = f.dim(), f.shape[0]
    dt = f.dtype
    nc = (n - 1) // 2 + 1
    _check(lib().mg_level_residual_restrict(dim, n, _dtype_code(f), _dptr(k, dt, f.shape, "k"),
                                            _dptr(u, dt, f.shape, "u"), _dptr(f, dt, None, "f"),
                                            _dptr(fc, dt, (nc,) * dim, "fc"), by, zchunk, _stream(stream)),
           "mg_level_residual_restrict")


def mg_level_smooth_restrict(u_in, f, u_out, fc, zchunk=4, order=0, stream=None) -> None:
    """Fused last pre-smoothing sweep + residual + full weighting (3D, float32 or float16)."""
    dim, n = f.dim(), f.shape[0]
    dt = f.dtype
    nc = (n - 1) // 2 + 1
    _check(lib().mg_level_smooth_restrict(dim, n, _dtype_code(f), _dptr(u_in, dt, f.shape, "u_in"),
                                          _dptr(f, dt, f.shape, "f"), _dptr(u_out, dt, f.shape, "u_out"),
                                          _dptr(fc, dt, (nc,) * dim, "fc"), int(zchunk), int(order),
                                          _stream(stream)), "mg_level_smooth_restrict")


def mg_level_smooth2_zero(f, u_out, by=12, zchunk=16, order=0, stream=None) -> None:
    """The first two red-first pre-smoothing sweeps from a zero iterate, fused (float32 or float16; 3D: by
    12 or 16 rows, zchunk planes per workgroup; 2D: by ignored, zchunk rows per wavefront)."""
    dim, n = f.dim(), f.shape[0]
    dt = f.dtype
    _check(lib().mg_level_smooth2_zero(dim, n, _dtype_code(f), _dptr(f, dt, f.shape, "f"),
                                       _dptr(u_out, dt, f.shape, "u_out"), int(by), int(zchunk), int(order),
                                       _stream(stream)), "mg_level_smooth2_zero")


def mg_level_smooth2_correct(u_in, f, ec, u_out, smoother=SMOOTH_RBGS, zchunk=32, order=0, stream=None) -> None:
    """The coarse-grid correction and the first two post-smoothing sweeps, fused (2D, float32 or float16;
    smoother SMOOTH_RBGS red first or SMOOTH_RBGS_SYM black first)."""
    dim, n = f.dim(), f.shape[0]
    dt = f.dtype
    nc = (n - 1) // 2 + 1
    _check(lib().mg_level_smooth2_correct(dim, n, _dtype_code(f), int(smoother), _dptr(u_in, dt, f.shape, "u_in"),
                                          _dptr(f, dt, f.shape, "f"), _dptr(ec, dt, (nc,) * dim, "ec"),
                                          _dptr(u_out, dt, f.shape, "u_out"), int(zchunk), int(order),
                                          _stream(stream)), "mg_level_smooth2_correct")


def mg_level_prolong_correct(u, ec, stream=None) -> None:
    dim, n = u.dim(), u.shape[0]
    dt = u.dtype
    nc = (n - 1) // 2 + 1
    _check(lib().mg_level_prolong_correct(dim, n, _dtype_code(u), _dptr(u, dt, None, "u"),
                                          _dptr(ec, dt, (nc,) * dim, "ec"), _stream(stream)),
           "mg_level_prolong_correct")


def mg_level_coarsest(u, f, k=None, stream=None) -> None:
    dim = f.dim()
    dt = f.dtype
    _check(lib().mg_level_coarsest(dim, _dtype_code(f), _dptr(k, dt, (3,) * dim, "k"), _dptr(u, dt, (3,) * dim, "u"),
                                   _dptr(f, dt, (3,) * dim, "f"), _stream(stream)), "mg_level_coarsest")


def mg_level_coarsest_cg(u, f, k=None, iters=0, stream=None) -> None:
    """Conjugate gradients on a coarsest grid (any n = 2^c + 1 within the limits), from u = 0."""
    dim, n = f.dim(), f.shape[0]
    dt = f.dtype
    _check(lib().mg_level_coarsest_cg(dim, n, _dtype_code(f), _dptr(k, dt, f.shape, "k"), _dptr(u, dt, f.shape, "u"),
                                      _dptr(f, dt, f.shape, "f"), int(iters), _stream(stream)), "mg_level_coarsest_cg")


# constant stencil (FP64, node grids): host stencil of 2*dim + 1 coefficients
def _st_host(stencil, dim):
    vals = [float(x) for x in stencil]
    if len(vals) != 2 * dim + 1:
        raise ValueError(f"a {dim}D stencil has {2 * dim + 1} coefficients")
    return (C.c_double * len(vals))(*vals)


def mg_level_st_smooth(u_in, f, u_out, stencil, smoother=SMOOTH_RBGS, omega=0.0, stream=None) -> None:
    import torch

    dim, n = f.dim(), f.shape[0]
    _check(lib().mg_level_st_smooth(dim, n, _st_host(stencil, dim), smoother, float(omega),
                                    _dptr(u_in, torch.float64, f.shape, "u_in"), _dptr(f, torch.float64, None, "f"),
                                    _dptr(u_out, torch.float64, f.shape, "u_out"), _stream(stream)),
           "mg_level_st_smooth")


def mg_level_st_residual_restrict(u, f, fc, stencil, stream=None) -> None:
    import torch

    dim, n = f.dim(), f.shape[0]
    nc = (n - 1) // 2 + 1
    _check(lib().mg_level_st_residual_restrict(dim, n, _st_host(stencil, dim), _dptr(u, torch.float64, f.shape, "u"),
                                               _dptr(f, torch.float64, None, "f"),
                                               _dptr(fc, torch.float64, (nc,) * dim, "fc"), _stream(stream)),
           "mg_level_st_residual_restrict")


def mg_level_st_coarsest(u, f, stencil, stream=None) -> None:
    import torch

    dim = f.dim()
    _check(lib().mg_level_st_coarsest(dim, _st_host(stencil, dim), _dptr(u, torch.float64, (3,) * dim, "u"),
                                      _dptr(f, torch.float64, (3,) * dim, "f"), _stream(stream)),
           "mg_level_st_coarsest")


# complex diffusion (FP64 complex, n = 2^L cells per axis, Neumann boundary)
def mg_cdiff_setup(dim, n, tau, theta=math.pi / 30, k=1.0, smoother=SMOOTH_RBGS, omega=0.0, nu1=2, nu2=2,
                   stream=None) -> int:
    """Context for the implicit-Euler FAS solver of the complex diffusion equation."""
    cp = _CDiffParams(int(dim), int(n), float(tau), float(theta), float(k), int(smoother), float(omega), int(nu1),
                      int(nu2))
    out = C.c_void_p()
    _check(lib().mg_cdiff_setup(C.byref(cp), _stream(stream), C.byref(out)), "mg_cdiff_setup")
    return _track(out.value)


def _cd_ptr(t, name):
    """Device pointer of a contiguous complex128 tensor ((re, im) FP64 pairs)."""
    import torch

    return _dptr(t, torch.complex128, None, name)


def mg_cdiff_fas(ctx: int, u, f) -> None:
    """One FAS cycle on u (complex128, in place) for N(u) = f."""
    if u.shape != f.shape:
        raise ValueError("u and f must have the same shape")
    _check(lib().mg_cdiff_fas(ctx, _cd_ptr(u, "u"), _cd_ptr(f, "f")), "mg_cdiff_fas")


def mg_cdiff_apply(ctx: int, u, out) -> None:
    """out = N(u) = u / tau - div(g(Im u) grad u)."""
    if u.shape != out.shape:
        raise ValueError("u and out must have the same shape")
    _check(lib().mg_cdiff_apply(ctx, _cd_ptr(u, "u"), _cd_ptr(out, "out")), "mg_cdiff_apply")


def mg_cdiff_run(ctx: int, u, steps: int, tol: float = 1e-5, max_cycles: int = 20):
    """Implicit-Euler steps on u (in place).  Returns (status, [cycles per step],
    [[residual norms] per step])."""
    nc = (C.c_int * max(1, steps))()
    hist = (C.c_double * max(1, steps * (max_cycles + 1)))()
    st = lib().mg_cdiff_run(ctx, _cd_ptr(u, "u"), int(steps), float(tol), int(max_cycles), nc, hist)
    _check(st, "mg_cdiff_run", ok=(MG_OK, MG_ENOTCONV))
    w = max_cycles + 1
    return st, list(nc)[:steps], [list(hist[m * w:m * w + nc[m] + 1]) for m in range(steps)]


# cell-centred Neumann grids (FP64, n = 2^L cells per axis)
def mg_level_cc_smooth(u_in, f, u_out, smoother=SMOOTH_RBGS, omega=0.0, stream=None) -> None:
    import torch

    dim, n = f.dim(), f.shape[0]
    _check(lib().mg_level_cc_smooth(dim, n, smoother, float(omega), _dptr(u_in, torch.float64, f.shape, "u_in"),
                                    _dptr(f, torch.float64, None, "f"), _dptr(u_out, torch.float64, f.shape, "u_out"),
                                    _stream(stream)), "mg_level_cc_smooth")


def mg_level_cc_residual_restrict(u, f, fc, stream=None) -> None:
    import torch

    dim, n = f.dim(), f.shape[0]
    _check(lib().mg_level_cc_residual_restrict(dim, n, _dptr(u, torch.float64, f.shape, "u"),
                                               _dptr(f, torch.float64, None, "f"),
                                               _dptr(fc, torch.float64, (n // 2,) * dim, "fc"), _stream(stream)),
           "mg_level_cc_residual_restrict")


def mg_level_cc_prolong_correct(u, ec, stream=None) -> None:
    import torch

    dim, n = u.dim(), u.shape[0]
    _check(lib().mg_level_cc_prolong_correct(dim, n, _dptr(u, torch.float64, None, "u"),
                                             _dptr(ec, torch.float64, (n // 2,) * dim, "ec"), _stream(stream)),
           "mg_level_cc_prolong_correct")


def mg_level_cc_remove_mean(v, stream=None) -> float:
    import torch

    dim, n = v.dim(), v.shape[0]
    out = C.c_double(0.0)
    _check(lib().mg_level_cc_remove_mean(dim, n, _dptr(v, torch.float64, None, "v"), C.byref(out), _stream(stream)),
           "mg_level_cc_remove_mean")
    return out.value


def mg_level_ir_update(u_in, e, f, u_out, r, k=None, by=0, zchunk=0, prefetch=0, waves=0, pairs=0,
                       stream=None, noalloc=False) -> float:
    """FP64 refinement pass; noalloc selects mg_level_ir_update_noalloc (static scratch)."""
    import torch

    dim, n = f.dim(), f.shape[0]
    sh = f.shape
    out = C.c_double(0.0)
    fn = lib().mg_level_ir_update_noalloc if noalloc else lib().mg_level_ir_update
    _check(fn(dim, n, _dptr(k, torch.float64, sh, "k"), _dptr(u_in, torch.float64, sh, "u_in"),
                                    _dptr(e, torch.float32, sh, "e"), _dptr(f, torch.float64, sh, "f"),
                                    _dptr(u_out, torch.float64, sh, "u_out"), _dptr(r, torch.float32, sh, "r"),
                                    C.byref(out), by, zchunk, prefetch, waves, pairs, _stream(stream)),
           "mg_level_ir_update_noalloc" if noalloc else "mg_level_ir_update")
    return out.value


def mg_level_ir_update_f16(u_in, e16, e_scale, prev_max, f, u_out, r16, by=0, zchunk=0, prefetch=0, waves=0,
                           stream=None):
    """Refinement pass of the binary16 form; e16 None: no update.  Returns (||r||, max |r|)."""
    import torch

    dim, n = f.dim(), f.shape[0]
    sh = f.shape
    nrm, mx = C.c_double(0.0), C.c_double(0.0)
    _check(lib().mg_level_ir_update_f16(dim, n, _dptr(u_in, torch.float64, sh, "u_in"),
                                        _dptr(e16, torch.float16, sh, "e16"), float(e_scale), float(prev_max),
                                        _dptr(f, torch.float64, sh, "f"), _dptr(u_out, torch.float64, sh, "u_out"),
                                        _dptr(r16, torch.float16, sh, "r16"), C.byref(nrm), C.byref(mx), by, zchunk,
                                        prefetch, waves, _stream(stream)), "mg_level_ir_update_f16")
    return nrm.value, mx.value


def mg_prof_enable(ctx: int, on: bool = True) -> None:
    _check(lib().mg_prof_enable(ctx, int(on)), "mg_prof_enable")


def mg_prof_read(ctx: int, kernel: int = 0):
    """(launches, total ms) since the last read of the measured finest-level launches of a kernel
    (0: plain smoothing sweeps, 1: refinement / norm pass) in steps the solves really ran."""
    n = C.c_int(0)
    ms = C.c_double(0.0)
    _check(lib().mg_prof_read_kernel(ctx, kernel, C.byref(n), C.byref(ms)), "mg_prof_read_kernel")
    return n.value, ms.value


def mg_copy_kernel(dst, src, stream=None) -> None:
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy: size mismatch")
    _check(lib().mg_copy_kernel(_dptr(dst), _dptr(src), nbytes, _stream(stream)), "mg_copy_kernel")


class Solver:
    """Owns one context; convenience wrapper over the mg_* calls."""

    def __init__(self, params: Params, stream=None):
        self.params = params
        self.ctx = mg_setup(params, stream)

    def vcycle(self, u, f):
        mg_vcycle(self.ctx, u, f)

    def solve(self, u, f, tol=1e-8, max_cycles=50):
        return mg_solve(self.ctx, u, f, tol, max_cycles)

    def residual_norm(self, u, f):
        return mg_residual_norm(self.ctx, u, f)

    @property
    def num_levels(self):
        return mg_num_levels(self.ctx)

    def close(self):
        if self.ctx:
            mg_destroy(self.ctx)
            self.ctx = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # Only while the interpreter runs normally; at exit the registry's
        # shutdown() has already destroyed the context.
        try:
            if self.ctx and self.ctx in _live:
                self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- batches
def mg_batch_setup(params_list, stream=None) -> int:
    """One context for many instances (list of Params; FP32_IR, Laplacian)."""
    arr = (_Params * len(params_list))(*[p.to_c() for p in params_list])
    out = C.c_void_p()
    _check(lib().mg_batch_setup(len(params_list), arr, _stream(stream), C.byref(out)), "mg_batch_setup")
    return _track(out.value)


def mg_batch_solve(ctx: int, us, fs, tol: float = 1e-8, max_cycles: int = 50):
    """Solve every instance; returns (worst status, [cycles], [status])."""
    import torch

    n = len(us)
    up = (C.c_void_p * n)(*[_dptr(u, torch.float64, name="u") for u in us])
    fp = (C.c_void_p * n)(*[_dptr(f, torch.float64, name="f") for f in fs])
    cyc = (C.c_int * n)()
    stt = (C.c_int * n)()
    st = lib().mg_batch_solve(ctx, up, fp, float(tol), int(max_cycles), cyc, stt)
    _check(st, "mg_batch_solve", ok=(MG_OK, MG_ENOTCONV, MG_EDIVERGED))
    return st, list(cyc), list(stt)


# ----------------------------------------------------------------- serving
@dataclass
class ServerParams:
    hbm_budget_bytes: int = 64 << 30
    max_slots: int = 64
    max_n2d: int = 2049
    max_n3d: int = 257
    smoother: int = SMOOTH_RBGS
    omega: float = 0.0
    nu1: int = 2
    nu2: int = 2
    tol: float = 1e-8
    max_cycles: int = 50

    def to_c(self):
        return _ServerParams(self.hbm_budget_bytes, self.max_slots, self.max_n2d, self.max_n3d, self.smoother,
                             self.omega, self.nu1, self.nu2, self.tol, self.max_cycles)


def mg_server_create(sp: ServerParams, stream=None) -> int:
    cp = sp.to_c()
    out = C.c_void_p()
    _check(lib().mg_server_create(C.byref(cp), _stream(stream), C.byref(out)), "mg_server_create")
    return _track(out.value)


def mg_server_submit(ctx: int, f_host) -> int:
    """Queue a request; f_host is a C-contiguous float64 numpy array of shape (n,)*dim."""
    import numpy as np

    f = np.ascontiguousarray(f_host, dtype=np.float64)
    rid = C.c_longlong(0)
    _check(lib().mg_server_submit(ctx, f.ndim, f.shape[0], f.ctypes.data, C.byref(rid)), "mg_server_submit")
    _server_shapes[(ctx, rid.value)] = f.shape
    return rid.value


def mg_server_submit_device(ctx: int, f_dev, u_dev) -> int:
    """Queue a request fed from device memory: f_dev (float64 tensor on the
    device, left unchanged until the request is done) is copied device to
    device at admission; the solution lands in u_dev (same shape) when
    mg_server_poll reports the request."""
    import torch

    if tuple(u_dev.shape) != tuple(f_dev.shape):
        raise ValueError("u_dev and f_dev must have the same shape")
    rid = C.c_longlong(0)
    _check(lib().mg_server_submit_device(ctx, f_dev.dim(), f_dev.shape[0], _dptr(f_dev, torch.float64, None, "f_dev"),
                                         _dptr(u_dev, torch.float64, None, "u_dev"), C.byref(rid)),
           "mg_server_submit_device")
    return rid.value


_server_shapes = {}  # (server, request id) -> shape of the request's grid


def mg_server_step(ctx: int):
    """Admit + one refinement step of every active request; returns (active, queued)."""
    a, q = C.c_int(0), C.c_int(0)
    _check(lib().mg_server_step(ctx, C.byref(a), C.byref(q)), "mg_server_step")
    return a.value, q.value


def mg_server_poll(ctx: int, cap: int = 4096):
    ids = (C.c_longlong * cap)()
    nd = C.c_int(0)
    _check(lib().mg_server_poll(ctx, ids, cap, C.byref(nd)), "mg_server_poll")
    return list(ids[: nd.value])


def mg_server_fetch(ctx: int, req_id: int, shape=None, out=None):
    """(status, u or None, cycles, final relative residual, latency seconds).

    The solution is copied into `out` (a C-contiguous float64 array of the
    request's shape) when given, else into a new array when `shape` is given."""
    import numpy as np

    u = out if out is not None else (np.empty(shape, dtype=np.float64) if shape is not None else None)
    if u is not None and (u.dtype != np.float64 or not u.flags.c_contiguous or not u.flags.writeable):
        raise ValueError("out must be a writeable C-contiguous float64 array")
    if u is not None and _server_shapes.get((ctx, req_id), u.shape) != u.shape:
        raise ValueError(f"output shape {u.shape} != request shape {_server_shapes[(ctx, req_id)]}")
    cyc, rr, lat = C.c_int(0), C.c_double(0.0), C.c_double(0.0)
    st = lib().mg_server_fetch(ctx, req_id, u.ctypes.data if u is not None else None, C.byref(cyc), C.byref(rr),
                               C.byref(lat))
    _check(st, "mg_server_fetch", ok=(MG_OK, MG_ENOTCONV, MG_EDIVERGED))
    _server_shapes.pop((ctx, req_id), None)
    return st, u, cyc.value, rr.value, lat.value


def mg_server_info(ctx: int):
    used, a, q = C.c_size_t(0), C.c_int(0), C.c_int(0)
    _check(lib().mg_server_info(ctx, C.byref(used), C.byref(a), C.byref(q)), "mg_server_info")
    return used.value, a.value, q.value
