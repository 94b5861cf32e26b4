"""Plain CPU reference (oracle) of the geometric multigrid V-cycle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The product package never imports it.

The arithmetic lives in ``oracle.cpp`` (plain loops, FP64 / FP32, no
floating-point contraction, optional OpenMP over the outermost loop).  This
module only builds/loads that library and marshals numpy arrays into it.
Every array is a C-ordered numpy array of shape (n, n) or (n, n, n), x fastest,
boundary included.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the loader at a deliberately mutated build of oracle.cpp.
_LIB_OVERRIDE = os.environ.get("MG_ORACLE_LIB")

CXXFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

SMOOTH_RBGS = 0
SMOOTH_JACOBI = 1
SMOOTH_RBGS_SYM = 2  # symmetric red-black: red first before the correction, black first after it
CYCLE_V, CYCLE_W, CYCLE_F = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.run(["g++", *CXXFLAGS, _SRC, "-o", tmp], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = C.c_double
_i = C.c_int
_p = C.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = C.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
    sig = {
        "orc_num_threads": (_i, []),
        "orc_residual_f64": (None, [_i, _i, _p, _p, _p, _p]),
        "orc_residual_f32": (None, [_i, _i, _p, _p, _p, _p]),
        "orc_smooth_f64": (None, [_i, _i, _p, _i, _d, _p, _p]),
        "orc_smooth_f32": (None, [_i, _i, _p, _i, _d, _p, _p]),
        "orc_rbgs_colour_f64": (None, [_i, _i, _p, _d, _i, _i, _p, _p]),
        "orc_restrict_f64": (None, [_i, _i, _p, _p]),
        "orc_restrict_f32": (None, [_i, _i, _p, _p]),
        "orc_prolong_correct_f64": (None, [_i, _i, _p, _p]),
        "orc_prolong_correct_f32": (None, [_i, _i, _p, _p]),
        "orc_coarsest_f64": (None, [_i, _p, _p, _p]),
        "orc_residual_norm_f64": (_d, [_i, _i, _p, _p, _p]),
        "orc_vcycle_f64": (_i, [_i, _i, _p, _i, _d, _i, _i, _p, _p]),
        "orc_vcycle_f32": (_i, [_i, _i, _p, _i, _d, _i, _i, _p, _p]),
        "orc_cycle_f64": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p]),
        "orc_cycle_f32": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p]),
        "orc_coarsest_cg_f64": (None, [_i, _i, _p, _i, _p, _p]),
        "orc_coarsest_cg_f32": (None, [_i, _i, _p, _i, _p, _p]),
        "orc_solve_f64": (_i, [_i, _i, _p, _i, _d, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_solve_mg_f64": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_ir_update_f32": (_d, [_i, _i, _p, _p, _p, _p, _p]),
        "orc_solve_ir_f32": (_i, [_i, _i, _p, _i, _d, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_solve_ir_mg_f32": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_half_from_float": (None, [_p, _p, C.c_longlong]),
        "orc_half_to_float": (None, [_p, _p, C.c_longlong]),
        "orc_residual_f16": (None, [_i, _i, _p, _p, _p, _p]),
        "orc_smooth_f16": (None, [_i, _i, _p, _i, _d, _p, _p]),
        "orc_restrict_f16": (None, [_i, _i, _p, _p]),
        "orc_prolong_correct_f16": (None, [_i, _i, _p, _p]),
        "orc_cycle_f16": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p]),
        "orc_fp16_scale": (_d, [_d]),
        "orc_ir_update_f16": (_d, [_i, _i, _p, _p, _p, _d, _p, _d, _p, _p]),
        "orc_solve_ir_mg_f16": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_cc_residual": (None, [_i, _i, _p, _p, _p]),
        "orc_cc_smooth": (None, [_i, _i, _i, _d, _p, _p]),
        "orc_cc_restrict": (None, [_i, _i, _p, _p]),
        "orc_cc_prolong_correct": (None, [_i, _i, _p, _p]),
        "orc_cc_sum": (_d, [_i, _i, _p]),
        "orc_cc_residual_norm": (_d, [_i, _i, _p, _p]),
        "orc_cc_cycle": (_i, [_i, _i, _i, _d, _i, _i, _i, _p, _p]),
        "orc_cc_solve": (_i, [_i, _i, _i, _d, _i, _i, _i, _p, _p, _d, _i, _p, _p, _p]),
        "orc_st_residual": (None, [_i, _i, _p, _p, _p, _p]),
        "orc_st_smooth": (None, [_i, _i, _p, _i, _d, _p, _p]),
        "orc_st_coarsest": (None, [_i, _p, _p, _p]),
        "orc_st_residual_norm": (_d, [_i, _i, _p, _p, _p]),
        "orc_st_solve": (_i, [_i, _i, _p, _i, _d, _i, _i, _i, _p, _p, _d, _i, _p, _p]),
        "orc_cd_apply": (None, [_i, _i, _d, _d, _d, _d, _d, _p, _p]),
        "orc_cd_g": (None, [_i, _i, _d, _d, _d, _d, _p, _p]),
        "orc_cd_sweep": (None, [_i, _i, _d, _d, _d, _d, _d, _i, _d, _p, _p]),
        "orc_cd_residual_norm": (_d, [_i, _i, _d, _d, _d, _d, _d, _p, _p]),
        "orc_cd_fas": (_i, [_i, _i, _d, _d, _d, _d, _d, _i, _d, _i, _i, _p, _p]),
        "orc_cd_run": (_i, [_i, _i, _d, _d, _d, _d, _d, _i, _d, _i, _i, _p, _i, _d, _i, _p, _p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _chk(a, dtype, name):
    if a is None:
        return None
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError(f"{name} must be a C-contiguous {np.dtype(dtype).name} numpy array")
    return a


def _dims(a):
    dim = a.ndim
    n = a.shape[0]
    if dim not in (2, 3) or any(s != n for s in a.shape):
        raise ValueError(f"expected a square/cubic node array, got shape {a.shape}")
    return dim, n


def num_threads() -> int:
    return _load().orc_num_threads()


def residual(u, f, k=None):
    """r = f - A u on inner nodes, 0 on the boundary (FP64 or FP32 by dtype;
    float16 u, f give a float32 residual computed in float, k float32)."""
    dt = u.dtype
    if dt == np.float16:
        _chk(u, dt, "u"), _chk(f, dt, "f"), _chk(k, np.float32, "k")
        dim, n = _dims(u)
        r = np.zeros(u.shape, dtype=np.float32)
        _load().orc_residual_f16(dim, n, _ptr(k), _ptr(u), _ptr(f), _ptr(r))
        return r
    _chk(u, dt, "u"), _chk(f, dt, "f"), _chk(k, dt, "k")
    dim, n = _dims(u)
    r = np.zeros_like(u)
    fn = _load().orc_residual_f64 if dt == np.float64 else _load().orc_residual_f32
    fn(dim, n, _ptr(k), _ptr(u), _ptr(f), _ptr(r))
    return r


def smooth(u, f, smoother=SMOOTH_RBGS, omega=1.0, k=None):
    """One smoothing sweep; returns a new array (float16: binary16 cells,
    float arithmetic, k float32)."""
    dt = u.dtype
    _chk(u, dt, "u"), _chk(f, dt, "f"), _chk(k, np.float32 if dt == np.float16 else dt, "k")
    dim, n = _dims(u)
    out = u.copy()
    fn = {np.dtype(np.float64): _load().orc_smooth_f64, np.dtype(np.float32): _load().orc_smooth_f32,
          np.dtype(np.float16): _load().orc_smooth_f16}[dt]
    fn(dim, n, _ptr(k), smoother, omega, _ptr(out), _ptr(f))
    return out


def rbgs_colour(u, f, colour, omega=1.0, reverse=False, k=None):
    """Red (0) or black (1) half-sweep with serial loops, optionally reversed."""
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u)
    out = u.copy()
    _load().orc_rbgs_colour_f64(dim, n, _ptr(k), omega, colour, int(reverse), _ptr(out), _ptr(f))
    return out


def restrict(r, out_dtype=None):
    """Full-weighting restriction of a fine residual to the next coarser grid
    (out_dtype float16: a float32 residual restricted in float into binary16
    cells)."""
    dt = r.dtype
    _chk(r, dt, "r")
    dim, nf = _dims(r)
    nc = (nf - 1) // 2 + 1
    if out_dtype is not None and np.dtype(out_dtype) == np.float16:
        _chk(r, np.float32, "r")
        fc = np.zeros((nc,) * dim, dtype=np.float16)
        _load().orc_restrict_f16(dim, nf, _ptr(r), _ptr(fc))
        return fc
    fc = np.zeros((nc,) * dim, dtype=dt)
    fn = _load().orc_restrict_f64 if dt == np.float64 else _load().orc_restrict_f32
    fn(dim, nf, _ptr(r), _ptr(fc))
    return fc


def prolong_correct(u, ec):
    """u + P ec on inner fine nodes (bi-/trilinear interpolation); returns a new array."""
    dt = u.dtype
    _chk(u, dt, "u"), _chk(ec, dt, "ec")
    dim, nf = _dims(u)
    if ec.shape != ((nf - 1) // 2 + 1,) * dim:
        raise ValueError("coarse array has the wrong shape")
    out = u.copy()
    fn = {np.dtype(np.float64): _load().orc_prolong_correct_f64, np.dtype(np.float32): _load().orc_prolong_correct_f32,
          np.dtype(np.float16): _load().orc_prolong_correct_f16}[dt]
    fn(dim, nf, _ptr(out), _ptr(ec))
    return out


def coarsest(u, f, k=None):
    """Exact solve on the n = 3 grid; returns a new array."""
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u)
    if n != 3:
        raise ValueError("coarsest solve needs n = 3")
    out = u.copy()
    _load().orc_coarsest_f64(dim, _ptr(k), _ptr(out), _ptr(f))
    return out


def residual_norm(u, f, k=None) -> float:
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u)
    return float(_load().orc_residual_norm_f64(dim, n, _ptr(k), _ptr(u), _ptr(f)))


def coarsest_cg(u, f, k=None, iters=0):
    """Conjugate gradients on a coarsest grid (any n = 2^L+1) from u = 0, `iters`
    steps (0: 4(n-1)); FP64 or FP32 by dtype; returns a new array (u is only
    used for its shape)."""
    dt = f.dtype
    _chk(u, dt, "u"), _chk(f, dt, "f"), _chk(k, dt, "k")
    dim, n = _dims(f)
    out = np.zeros_like(f)
    fn = _load().orc_coarsest_cg_f64 if dt == np.float64 else _load().orc_coarsest_cg_f32
    fn(dim, n, _ptr(k), int(iters), _ptr(out), _ptr(f))
    return out


def vcycle(u, f, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, k=None, cycle=CYCLE_V, coarse_n=3, cg_iters=0):
    """One multigrid cycle (V by default; W, F with `cycle`; coarsest level of
    edge `coarse_n`, solved by conjugate gradients when larger than 3);
    FP64 or FP32 by dtype; returns a new array."""
    dt = u.dtype
    _chk(u, dt, "u"), _chk(f, dt, "f"), _chk(k, np.float32 if dt == np.float16 else dt, "k")
    dim, n = _dims(u)
    out = u.copy()
    fn = {np.dtype(np.float64): _load().orc_cycle_f64, np.dtype(np.float32): _load().orc_cycle_f32,
          np.dtype(np.float16): _load().orc_cycle_f16}[dt]
    rc = fn(dim, n, _ptr(k), smoother, omega, nu1, nu2, cycle, coarse_n, cg_iters, _ptr(out), _ptr(f))
    if rc != 0:
        raise ValueError(f"oracle cycle rejected its arguments (rc={rc})")
    return out


def solve(u0, f, tol=1e-8, max_cycles=50, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, k=None, cycle=CYCLE_V,
          coarse_n=3, cg_iters=0):
    """FP64 multigrid solve.  Returns (u, history of ||f - A u||_2, status)."""
    _chk(u0, np.float64, "u0"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u0)
    u = u0.copy()
    hist = np.zeros(max_cycles + 1)
    cyc = C.c_int(0)
    rc = _load().orc_solve_mg_f64(dim, n, _ptr(k), smoother, omega, nu1, nu2, cycle, coarse_n, cg_iters, _ptr(u),
                                  _ptr(f), tol, max_cycles, _ptr(hist), C.addressof(cyc))
    if rc < 0:
        raise ValueError(f"oracle solve rejected its arguments (rc={rc})")
    return u, hist[: cyc.value + 1].copy(), rc


def ir_update(u, e, f, k=None):
    """One FP64 refinement pass: returns (u + e, float32 residual, ||r||)."""
    _chk(u, np.float64, "u"), _chk(e, np.float32, "e"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u)
    out = u.copy()
    r32 = np.zeros(u.shape, dtype=np.float32)
    rho = _load().orc_ir_update_f32(dim, n, _ptr(k), _ptr(out), _ptr(e), _ptr(f), _ptr(r32))
    return out, r32, float(rho)


def solve_ir_f32(u0, f, tol=1e-8, max_cycles=50, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, k=None,
                 cycle=CYCLE_V, coarse_n=3, cg_iters=0):
    """FP32 cycles inside FP64 iterative refinement.  Returns (u, history, status)."""
    _chk(u0, np.float64, "u0"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u0)
    u = u0.copy()
    hist = np.zeros(max_cycles + 1)
    cyc = C.c_int(0)
    rc = _load().orc_solve_ir_mg_f32(dim, n, _ptr(k), smoother, omega, nu1, nu2, cycle, coarse_n, cg_iters,
                                     _ptr(u), _ptr(f), tol, max_cycles, _ptr(hist), C.addressof(cyc))
    if rc < 0:
        raise ValueError(f"oracle solve rejected its arguments (rc={rc})")
    return u, hist[: cyc.value + 1].copy(), rc


def half_from_float(x):
    """float32 array -> nearest binary16 values (ties to even), as numpy float16."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.float16)
    _load().orc_half_from_float(_ptr(x), _ptr(out), x.size)
    return out


def half_to_float(h):
    h = np.ascontiguousarray(h, dtype=np.float16)
    out = np.zeros(h.shape, dtype=np.float32)
    _load().orc_half_to_float(_ptr(h), _ptr(out), h.size)
    return out


def fp16_scale(mx: float) -> float:
    """Power of two s with 8 <= s*mx < 16, exponent within -126..127 (1 for mx zero or not finite)."""
    return float(_load().orc_fp16_scale(float(mx)))


def ir_update_f16(u, e16, s_prev, f, s_next, k=None):
    """One FP64 refinement pass of the half-precision form.  e16 (float16, the
    correction scaled by s_prev) may be None (no update).  Returns (u_new,
    r16 = half(float(s_next) * float(r)), ||r||_2, max |r|)."""
    _chk(u, np.float64, "u"), _chk(e16, np.float16, "e16"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u)
    out = u.copy()
    r16 = np.zeros(u.shape, dtype=np.float16)
    mx = C.c_double(0.0)
    rho = _load().orc_ir_update_f16(dim, n, _ptr(k), _ptr(out), _ptr(e16), float(s_prev), _ptr(f), float(s_next),
                                    _ptr(r16), C.addressof(mx))
    return out, r16, float(rho), float(mx.value)


def solve_ir_f16(u0, f, tol=1e-8, max_cycles=50, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, k=None,
                 cycle=CYCLE_V, coarse_n=3, cg_iters=0):
    """Half-precision-storage cycles (float arithmetic) inside FP64 iterative
    refinement, with a power-of-two residual scale per step.  Returns (u,
    history, status); status -5 if the residual turns non-finite or grows
    1e6-fold."""
    _chk(u0, np.float64, "u0"), _chk(f, np.float64, "f"), _chk(k, np.float64, "k")
    dim, n = _dims(u0)
    u = u0.copy()
    hist = np.zeros(max_cycles + 1)
    cyc = C.c_int(0)
    rc = _load().orc_solve_ir_mg_f16(dim, n, _ptr(k), smoother, omega, nu1, nu2, cycle, coarse_n, cg_iters,
                                     _ptr(u), _ptr(f), tol, max_cycles, _ptr(hist), C.addressof(cyc))
    if rc == -1:
        raise ValueError(f"oracle solve rejected its arguments (rc={rc})")
    return u, hist[: cyc.value + 1].copy(), rc


# ------------------------------------------------------------------ cell-centred Neumann grids
# Arrays hold the n^dim cell values (n = 2^L cells per axis, h = 1/n), x fastest.


def _cc_dims(a):
    dim = a.ndim
    n = a.shape[0]
    if dim not in (2, 3) or any(s != n for s in a.shape) or n < 1 or (n & (n - 1)):
        raise ValueError(f"expected a square/cubic cell array of 2^L cells per axis, got shape {a.shape}")
    return dim, n


def cc_residual(u, f):
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _cc_dims(u)
    r = np.zeros_like(u)
    _load().orc_cc_residual(dim, n, _ptr(u), _ptr(f), _ptr(r))
    return r


def cc_smooth(u, f, smoother=SMOOTH_RBGS, omega=1.0):
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _cc_dims(u)
    out = u.copy()
    _load().orc_cc_smooth(dim, n, smoother, omega, _ptr(out), _ptr(f))
    return out


def cc_restrict(r):
    _chk(r, np.float64, "r")
    dim, nf = _cc_dims(r)
    fc = np.zeros((nf // 2,) * dim)
    _load().orc_cc_restrict(dim, nf, _ptr(r), _ptr(fc))
    return fc


def cc_prolong_correct(u, ec):
    _chk(u, np.float64, "u"), _chk(ec, np.float64, "ec")
    dim, nf = _cc_dims(u)
    if ec.shape != (nf // 2,) * dim:
        raise ValueError("coarse array has the wrong shape")
    out = u.copy()
    _load().orc_cc_prolong_correct(dim, nf, _ptr(out), _ptr(ec))
    return out


def cc_sum(u) -> float:
    _chk(u, np.float64, "u")
    dim, n = _cc_dims(u)
    return float(_load().orc_cc_sum(dim, n, _ptr(u)))


def cc_residual_norm(u, f) -> float:
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _cc_dims(u)
    return float(_load().orc_cc_residual_norm(dim, n, _ptr(u), _ptr(f)))


def cc_cycle(u, f, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, cycle=CYCLE_V):
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _cc_dims(u)
    out = u.copy()
    if _load().orc_cc_cycle(dim, n, smoother, omega, nu1, nu2, cycle, _ptr(out), _ptr(f)) != 0:
        raise ValueError("oracle cycle rejected its arguments")
    return out


def cc_solve(u0, f, tol=1e-8, max_cycles=50, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2, cycle=CYCLE_V):
    """Cell-centred Neumann solve (FP64).  Returns (u, history, status, projected f)."""
    _chk(u0, np.float64, "u0"), _chk(f, np.float64, "f")
    dim, n = _cc_dims(u0)
    u = u0.copy()
    hist = np.zeros(max_cycles + 1)
    fh = np.zeros_like(f)
    cyc = C.c_int(0)
    rc = _load().orc_cc_solve(dim, n, smoother, omega, nu1, nu2, cycle, _ptr(u), _ptr(f), tol, max_cycles,
                              _ptr(hist), C.addressof(cyc), _ptr(fh))
    if rc == -1:
        raise ValueError("oracle solve rejected its arguments")
    return u, hist[: cyc.value + 1].copy(), rc, fh


# ------------------------------------------------------------------ complex diffusion
# Complex cell arrays are numpy complex128 (re, im pairs), n = 2^L cells per axis.
# The diffusivity g(s) = e^{i theta} / (1 + (s / (k theta))^2) takes cos(theta)
# and sin(theta) as evaluated here (math.cos / math.sin), the same numbers the
# library's host code passes to its kernels.
import math as _math  # noqa: E402


class CD:
    """Parameters of the complex-diffusion problem."""

    def __init__(self, tau, theta=_math.pi / 30, k=1.0):
        self.tau, self.theta, self.k = float(tau), float(theta), float(k)
        self.ct, self.st = _math.cos(self.theta), _math.sin(self.theta)

    def args(self):
        return (self.tau, self.theta, self.k, self.ct, self.st)


def _cchk(a, name):
    return _chk(a, np.complex128, name)


def cd_apply(u, P: CD):
    """N(u) = u / tau - div(g(Im u) grad u) (cell-centred, Neumann)."""
    _cchk(u, "u")
    dim, n = _cc_dims(u)
    out = np.zeros_like(u)
    _load().orc_cd_apply(dim, n, *P.args(), _ptr(u), _ptr(out))
    return out


def cd_g(u, P: CD):
    _cchk(u, "u")
    dim, n = _cc_dims(u)
    g = np.zeros_like(u)
    _load().orc_cd_g(dim, n, P.theta, P.k, P.ct, P.st, _ptr(u), _ptr(g))
    return g


def cd_sweep(u, f, P: CD, smoother=SMOOTH_RBGS, omega=1.0):
    _cchk(u, "u"), _cchk(f, "f")
    dim, n = _cc_dims(u)
    out = u.copy()
    _load().orc_cd_sweep(dim, n, *P.args(), smoother, omega, _ptr(out), _ptr(f))
    return out


def cd_residual_norm(u, f, P: CD) -> float:
    _cchk(u, "u"), _cchk(f, "f")
    dim, n = _cc_dims(u)
    return float(_load().orc_cd_residual_norm(dim, n, *P.args(), _ptr(u), _ptr(f)))


def cd_fas(u, f, P: CD, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2):
    _cchk(u, "u"), _cchk(f, "f")
    dim, n = _cc_dims(u)
    out = u.copy()
    if _load().orc_cd_fas(dim, n, *P.args(), smoother, omega, nu1, nu2, _ptr(out), _ptr(f)) != 0:
        raise ValueError("oracle FAS cycle rejected its arguments")
    return out


def cd_run(u0, P: CD, steps=1, tol=1e-5, max_cycles=20, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2):
    """Implicit-Euler time steps with FAS per step.  Returns (u, cycles per step,
    residual histories per step (list of arrays), status)."""
    _cchk(u0, "u0")
    dim, n = _cc_dims(u0)
    u = u0.copy()
    cyc = np.zeros(max(steps, 1), dtype=np.int32)
    hist = np.zeros((max(steps, 1), max_cycles + 1))
    rc = _load().orc_cd_run(dim, n, *P.args(), smoother, omega, nu1, nu2, _ptr(u), steps, tol, max_cycles,
                            _ptr(cyc), _ptr(hist))
    if rc == -1:
        raise ValueError("oracle run rejected its arguments")
    return u, cyc[:steps].copy(), [hist[m, : cyc[m] + 1].copy() for m in range(steps)], rc


# ------------------------------------------------------------------ constant stencil
# A = (1/h^2) stencil on node-based Dirichlet grids (FP64); the stencil is a
# sequence of 2d+1 coefficients, centre first, then -x, +x, -y, +y[, -z, +z].
def _st(stencil, dim):
    a = np.ascontiguousarray(np.asarray(stencil, dtype=np.float64))
    if a.shape != (2 * dim + 1,):
        raise ValueError(f"a {dim}D stencil has {2 * dim + 1} coefficients")
    return a


def st_residual(u, f, stencil):
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _dims(u)
    a = _st(stencil, dim)
    r = np.zeros_like(u)
    _load().orc_st_residual(dim, n, _ptr(a), _ptr(u), _ptr(f), _ptr(r))
    return r


def st_smooth(u, f, stencil, smoother=SMOOTH_RBGS, omega=1.0):
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _dims(u)
    a = _st(stencil, dim)
    out = u.copy()
    _load().orc_st_smooth(dim, n, _ptr(a), smoother, omega, _ptr(out), _ptr(f))
    return out


def st_coarsest(f, stencil):
    _chk(f, np.float64, "f")
    dim, n = _dims(f)
    if n != 3:
        raise ValueError("the coarsest grid has n = 3")
    a = _st(stencil, dim)
    u = np.zeros_like(f)
    _load().orc_st_coarsest(dim, _ptr(a), _ptr(u), _ptr(f))
    return u


def st_residual_norm(u, f, stencil) -> float:
    _chk(u, np.float64, "u"), _chk(f, np.float64, "f")
    dim, n = _dims(u)
    a = _st(stencil, dim)
    return float(_load().orc_st_residual_norm(dim, n, _ptr(a), _ptr(u), _ptr(f)))


def st_solve(u0, f, stencil, tol=1e-8, max_cycles=50, smoother=SMOOTH_RBGS, omega=1.0, nu1=2, nu2=2,
             cycle=CYCLE_V):
    """FP64 multigrid solve with a constant stencil.  Returns (u, history, status)."""
    _chk(u0, np.float64, "u0"), _chk(f, np.float64, "f")
    dim, n = _dims(u0)
    a = _st(stencil, dim)
    u = u0.copy()
    hist = np.zeros(max_cycles + 1)
    cyc = C.c_int(0)
    rc = _load().orc_st_solve(dim, n, _ptr(a), smoother, omega, nu1, nu2, cycle, _ptr(u), _ptr(f), tol, max_cycles,
                              _ptr(hist), C.addressof(cyc))
    if rc < 0:
        raise ValueError(f"oracle solve rejected its arguments (rc={rc})")
    return u, hist[: cyc.value + 1].copy(), rc
