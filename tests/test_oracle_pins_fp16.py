"""Pins of the oracle's binary16 storage form.

The binary16 hierarchy stores every V-cycle field as IEEE binary16 and
computes in float.  Its pieces are pinned against things other than
themselves: the float -> binary16 rounding against numpy's float16
conversion (round to nearest, ties to even, subnormals, overflow), each
single operation against the pinned float operation followed by that
rounding, the refinement pass against the pinned FP64 residual and numpy
arithmetic, the scale rule against its definition, and the whole form
against the FP64 solution.
"""

import numpy as np
import pytest

import inputs
import oracle

RB, JAC = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float16).view(np.uint16)


def test_half_rounding_matches_numpy():
    rng = np.random.default_rng(7)
    mags = np.float32(2.0) ** rng.uniform(-30, 18, 200000).astype(np.float32)
    x = (rng.choice([-1.0, 1.0], 200000).astype(np.float32) * mags).astype(np.float32)
    # ties and boundaries: half-way points between neighbouring binary16 values
    h = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float32)
    mid = ((h[:-1].astype(np.float64) + h[1:].astype(np.float64)) / 2).astype(np.float32)
    edge = np.array([65504, 65519.996, 65520, 65536, 1e30, 2**-24, 2**-25, 1.5 * 2**-25, 2**-26, 2**-14,
                     2**-14 * (1 - 2**-11), 0.0, -0.0, np.inf, -np.inf], np.float32)
    allx = np.concatenate([x, mid, -mid, h, edge])
    with np.errstate(over="ignore"):
        ref = allx.astype(np.float16)
    assert np.array_equal(bits(oracle.half_from_float(allx)), bits(ref))


def test_half_decode_matches_numpy():
    every = np.arange(0, 65536, dtype=np.uint32).astype(np.uint16).view(np.float16)
    finite = every[np.isfinite(every)]
    assert np.array_equal(oracle.half_to_float(finite), finite.astype(np.float32))


def arrays16(dim, n, seed):
    c = float((n - 1) ** 2)
    u = (inputs.random_guess(dim, n, 500 + seed) * (8.0 / c)).astype(np.float16)
    f = (inputs.uniform_rhs(dim, n, 600 + seed) * 12.0).astype(np.float16)
    return u, f


@pytest.mark.parametrize("dim,n", [(2, 17), (2, 65), (3, 9), (3, 33)])
def test_fp16_residual_is_float_residual(dim, n):
    u, f = arrays16(dim, n, 1)
    r16 = oracle.residual(u, f)
    r32 = oracle.residual(u.astype(np.float32), f.astype(np.float32))
    assert r16.dtype == np.float32 and np.array_equal(r16, r32)


@pytest.mark.parametrize("dim,n", [(2, 17), (2, 65), (3, 9), (3, 33)])
def test_fp16_jacobi_is_rounded_float_jacobi(dim, n):
    """Jacobi reads old values only: the binary16 sweep is the float sweep of
    the same values, rounded."""
    u, f = arrays16(dim, n, 2)
    got = oracle.smooth(u, f, smoother=JAC, omega=0.8)
    ref = oracle.smooth(u.astype(np.float32), f.astype(np.float32), smoother=JAC, omega=0.8).astype(np.float16)
    assert np.array_equal(bits(got), bits(ref))


@pytest.mark.parametrize("dim,n", [(2, 17), (3, 17)])
def test_fp16_rbgs_black_half_reads_rounded_red(dim, n):
    """An RBGS sweep on binary16 cells: red nodes equal the rounded float red
    update; black nodes equal the rounded float update computed from the
    rounded red values (the red values are stored before black reads them)."""
    u, f = arrays16(dim, n, 3)
    got = oracle.smooth(u, f, smoother=RB)
    u32, f32 = u.astype(np.float32), f.astype(np.float32)
    full32 = oracle.smooth(u32, f32, smoother=RB)  # float red then black
    idx = np.indices(u.shape).sum(axis=0)
    inner = np.zeros(u.shape, bool)
    inner[(slice(1, -1),) * dim] = True
    red = inner & (idx % 2 == 0)
    black = inner & (idx % 2 == 1)
    # red: each red update reads only black (old) values and f, so it is the
    # float red update, rounded
    assert np.array_equal(bits(got[red]), bits(full32[red].astype(np.float16)))
    # black: the float black update from the binary16 red values (a float
    # sweep that relaxes black first, the second half of the symmetric
    # smoother, on an iterate holding the rounded red values)
    u_red = u32.copy()
    u_red[red] = got[red].astype(np.float32)
    again = oracle.smooth(u_red, f32, smoother=oracle.SMOOTH_RBGS_SYM)
    assert np.array_equal(bits(got[black]), bits(again[black].astype(np.float16)))


@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
def test_fp16_restrict_and_prolong_are_rounded_float_ops(dim, n):
    u, f = arrays16(dim, n, 4)
    r = oracle.residual(u, f)
    fc = oracle.restrict(r, out_dtype=np.float16)
    assert np.array_equal(bits(fc), bits(oracle.restrict(r).astype(np.float16)))
    nc = (n - 1) // 2 + 1
    ec = (inputs.random_guess(dim, nc, 40) * 1e-3).astype(np.float16)
    got = oracle.prolong_correct(u, ec)
    ref = oracle.prolong_correct(u.astype(np.float32), ec.astype(np.float32)).astype(np.float16)
    assert np.array_equal(bits(got), bits(ref))


def test_fp16_scale_definition():
    rng = np.random.default_rng(3)
    for mx in list(2.0 ** rng.uniform(-123, 130, 4000)) + [1.0, 8.0, 16.0, 0.5, 2.0**-123, 2.0**130 * (1 - 2**-52)]:
        s = oracle.fp16_scale(mx)
        m, e = np.frexp(s)
        assert m == 0.5  # a power of two
        assert 8.0 <= s * mx < 16.0
    # beyond that range the exponent stops at -126 / 127: s stays a normal float
    assert oracle.fp16_scale(2.0**-1074) == 2.0**127
    assert oracle.fp16_scale(1.7e308) == 2.0**-126
    for bad in [0.0, np.inf, np.nan, -1.0]:
        assert oracle.fp16_scale(bad) == 1.0


@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
def test_fp16_refinement_pass(dim, n):
    """u + e16 / s_prev exactly, then the residual (pinned FP64 operator) scaled
    by s_next in float and rounded to binary16; norm and max of that residual."""
    u = inputs.random_guess(dim, n, 5)
    f = inputs.uniform_rhs(dim, n, 6)
    e16 = (inputs.random_guess(dim, n, 7) * 9.0).astype(np.float16)
    s_prev, s_next = 2.0**12, 2.0**-3
    u_new, r16, rho, mx = oracle.ir_update_f16(u, e16, s_prev, f, s_next)
    inner = (slice(1, -1),) * dim
    ref_u = u.copy()
    ref_u[inner] = u[inner] + e16[inner].astype(np.float64) / s_prev
    assert np.array_equal(u_new, ref_u)
    r64 = oracle.residual(ref_u, f)
    ref_r16 = (np.float32(s_next) * r64.astype(np.float32)).astype(np.float16)
    assert np.array_equal(bits(r16[inner]), bits(ref_r16[inner]))
    assert mx == np.abs(r64[inner]).max()
    assert rho == pytest.approx(np.linalg.norm(r64[inner]), rel=1e-14)
    # without a correction the iterate is unchanged
    u_same, _, rho0, _ = oracle.ir_update_f16(u, None, 1.0, f, s_next)
    assert np.array_equal(u_same, u)
    assert rho0 == pytest.approx(np.linalg.norm(oracle.residual(u, f)[inner]), rel=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 65), (3, 17)])
def test_fp16_cycle_tracks_fp32_cycle(dim, n):
    """One cycle on a residual of the size the refinement hands it: the
    binary16 correction agrees with the float one to a few binary16 ulps
    (relative 1e-2 in the 2-norm)."""
    f = inputs.uniform_rhs(dim, n, 8) * 12.0
    e32 = oracle.vcycle(np.zeros(f.shape, np.float32), f.astype(np.float32))
    e16 = oracle.vcycle(np.zeros(f.shape, np.float16), f.astype(np.float16))
    rel = np.linalg.norm(e16.astype(np.float64) - e32) / np.linalg.norm(e32)
    assert rel < 1e-2


@pytest.mark.parametrize("dim,n,smoother", [(2, 65, RB), (3, 33, RB), (3, 17, JAC)])
def test_fp16_refinement_reaches_fp64_solution(dim, n, smoother):
    omega = 1.0 if smoother == RB else 0.8
    f = inputs.uniform_rhs(dim, n, 9)
    u64, _, _ = oracle.solve(np.zeros_like(f), f, tol=1e-13, max_cycles=60, smoother=smoother, omega=omega)
    u16, h, rc = oracle.solve_ir_f16(np.zeros_like(f), f, tol=1e-12, max_cycles=80, smoother=smoother, omega=omega)
    assert rc == 0 and h[-1] <= 1e-12 * h[0]
    assert np.linalg.norm(u16 - u64) <= 1e-10 * np.linalg.norm(u64)


@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33), (3, 65)])
def test_fp16_refinement_converges_like_fp32(dim, n):
    """To 1e-8 the binary16 form needs at most two refinement steps more than
    the float form on these grids (measured: the same count)."""
    f = inputs.uniform_rhs(dim, n, 10)
    _, h32, rc32 = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
    _, h16, rc16 = oracle.solve_ir_f16(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
    assert rc32 == 0 and rc16 == 0
    assert len(h16) <= len(h32) + 2
