"""Parity of the binary16 form (MG_PREC_FP16_IR) with the CPU oracle.

Every V-cycle field is stored as IEEE binary16 and computed in FP32 on both
sides, with the same expressions, the same rounding points (each value the
method stores is rounded to binary16, also where a fused kernel keeps it in
registers) and no FMA contraction, so fields are compared bit for bit.  The
refinement pass scales the residual by a power of two taken from the previous
pass's largest |r| on both sides.  Norms are sums in different orders (1e-13
relative), solve histories 1e-12 relative per step.
"""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

RB, JAC = 0, 1


def mg():
    import paper_1406_5369_amd as m

    return m


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def same(a, b):
    """Bitwise equality (binary16 arrays compared as their bit patterns)."""
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    if a.dtype == np.float16:
        return np.array_equal(a.view(np.uint16), b.view(np.uint16))
    return np.array_equal(a, b)


def arrays16(dim, n, seed):
    """Iterate and right-hand side of the magnitudes the refinement hands a
    cycle: the scaled residual is O(10) and c * u about as large, so the
    iterate spans binary16's normal and (on fine grids) subnormal range."""
    c = float((n - 1) ** 2)
    u = (inputs.random_guess(dim, n, 500 + seed) * (8.0 / c)).astype(np.float16)
    f = (inputs.uniform_rhs(dim, n, 600 + seed) * 12.0).astype(np.float16)
    return u, f


SMOOTH16 = [
    # dim, n, by, zchunk, prefetch, waves
    (2, 5, 0, 0, 0, 0), (2, 33, 16, 0, 0, 0), (2, 129, 0, 0, 0, 0), (2, 257, 32, 0, 0, 0), (2, 513, 8, 0, 0, 0),
    (3, 5, 0, 0, 1, 0), (3, 9, 8, 1, 2, 0), (3, 17, 16, 3, 1, 8), (3, 33, 0, 0, 2, 0), (3, 65, 32, 7, 2, 8),
    (3, 65, 8, 64, 1, 0), (3, 129, 16, 33, 2, 8), (3, 129, 32, 16, 1, 4), (3, 65, 12, 9, 1, 1),
    (3, 129, 8, 13, 2, 1), (3, 257, 16, 40, 1, 8),
]


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", SMOOTH16)
@pytest.mark.parametrize("smoother", [RB, JAC])
@pytest.mark.parametrize("variant", ["plain", "zero", "fused"])
def test_fp16_sweep_bitwise(dim, n, by, zc, pd, wv, smoother, variant, dev_ok):
    """Plain sweep, sweep from a zero iterate, and the first post-smoothing
    sweep with the coarse-grid correction (rounded to binary16 before the
    sweep, as the oracle stores it), on binary16 fields."""
    u, f = arrays16(dim, n, n + 7 * smoother)
    omega = 1.0 if smoother == RB else 0.8
    ec = None
    if variant == "zero":
        expect = oracle.smooth(np.zeros_like(f), f, smoother=smoother, omega=omega)
    elif variant == "fused":
        nc = (n - 1) // 2 + 1
        ec = (inputs.random_guess(dim, nc, 70 + n) * (8.0 / (n - 1) ** 2)).astype(np.float16)
        expect = oracle.smooth(oracle.prolong_correct(u, ec), f, smoother=smoother, omega=omega)
    else:
        expect = oracle.smooth(u, f, smoother=smoother, omega=omega)
    out = dev(np.zeros_like(u))
    mg().mg_level_smooth(None if variant == "zero" else dev(u), dev(f), out, smoother=smoother, omega=omega,
                         ec=dev(ec) if ec is not None else None, zero_guess=variant == "zero", by=by, zchunk=zc,
                         prefetch=pd, waves=wv)
    assert same(host(out), expect)


@pytest.mark.parametrize("dim,n,by,zc", [(2, 5, 0, 0), (2, 65, 8, 0), (2, 257, 32, 0), (2, 1025, 16, 0),
                                         (3, 5, 0, 0), (3, 17, 8, 1), (3, 65, 0, 0), (3, 129, 32, 9),
                                         (3, 257, 16, 20)])
def test_fp16_residual_restrict_bitwise(dim, n, by, zc, dev_ok):
    """The residual stays in FP32 inside the kernel; the restricted value is
    stored in binary16."""
    u, f = arrays16(dim, n, 3)
    expect = oracle.restrict(oracle.residual(u, f), out_dtype=np.float16)
    nc = (n - 1) // 2 + 1
    fc = dev(np.zeros((nc,) * dim, dtype=np.float16))
    mg().mg_level_residual_restrict(dev(u), dev(f), fc, by=by, zchunk=zc)
    assert same(host(fc), expect)


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 257), (3, 5), (3, 33), (3, 129)])
def test_fp16_prolong_correct_bitwise(dim, n, dev_ok):
    u, _ = arrays16(dim, n, 9)
    nc = (n - 1) // 2 + 1
    ec = (inputs.random_guess(dim, nc, 99) * (8.0 / (n - 1) ** 2)).astype(np.float16)
    expect = oracle.prolong_correct(u, ec)
    ud = dev(u)
    mg().mg_level_prolong_correct(ud, dev(ec))
    assert same(host(ud), expect)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp16_coarsest_bitwise(dim, dev_ok):
    """n = 3: one unknown; the oracle's cycle on a 3-node grid is its coarsest solve."""
    f = np.zeros((3,) * dim, dtype=np.float16)
    f[(1,) * dim] = np.float16(3.7)
    expect = oracle.vcycle(np.zeros_like(f), f)
    ud = dev(np.zeros_like(f))
    mg().mg_level_coarsest(ud, dev(f))
    assert same(host(ud), expect)


def test_fp16_level_ops_reject_coefficients(dev_ok):
    u, f = arrays16(3, 17, 1)
    k = dev(np.ones(u.shape, np.float16))
    with pytest.raises(mg().MGError) as ei:
        mg().mg_level_smooth(dev(u), dev(f), dev(np.zeros_like(u)), k=k)
    assert ei.value.code == mg().MG_ENOTSUP


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", [(2, 5, 0, 1, 1, 0), (2, 65, 0, 8, 1, 0), (2, 257, 0, 32, 2, 0),
                                              (2, 1025, 0, 100, 2, 0), (3, 5, 8, 1, 1, 4), (3, 33, 8, 4, 1, 4),
                                              (3, 65, 16, 9, 2, 4), (3, 129, 16, 16, 2, 8), (3, 257, 32, 31, 1, 8),
                                              (3, 9, 16, 2, 2, 4)])
@pytest.mark.parametrize("update", [True, False])
def test_fp16_refinement_pass(dim, n, by, zc, pd, wv, update, dev_ok):
    """u_out = u_in + e16 / e_scale, r16 = half(float(s) float(f - A u)) with s
    from the previous pass's largest |r|, norm and largest |r| of this pass."""
    import torch

    u = inputs.random_guess(dim, n, 13)
    f = inputs.uniform_rhs(dim, n, 14)
    e16 = (inputs.random_guess(dim, n, 15) * 9.0).astype(np.float16) if update else None
    e_scale, prev_max = 2.0 ** 13, 3.1e-3 * (n - 1) ** 2
    s_next = oracle.fp16_scale(prev_max)
    u_exp, r_exp, rho_exp, mx_exp = oracle.ir_update_f16(u, e16, e_scale, f, s_next)
    uo = dev(np.zeros_like(u))
    r = torch.zeros(u.shape, dtype=torch.float16, device="cuda")
    rho, mx = mg().mg_level_ir_update_f16(dev(u), dev(e16) if update else None, e_scale, prev_max, dev(f), uo, r,
                                          by=by, zchunk=zc, prefetch=pd, waves=wv)
    if update:
        assert same(host(uo), u_exp)
    assert same(host(r), r_exp)
    assert rho == pytest.approx(rho_exp, rel=1e-13)
    assert mx == mx_exp


# ---------------------------------------------------------------- full solves
def solve16(dim, n, f, smoother=RB, tol=1e-8, max_cycles=30, u0=None):
    m = mg()
    s = m.Solver(m.Params(dim=dim, n=n, smoother=smoother, precision=m.PREC_FP16_IR))
    u = dev(np.zeros_like(f) if u0 is None else u0)
    st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
    out = host(u)
    s.close()
    return st, cyc, np.array(hist), out


@pytest.mark.parametrize("dim,n,smoother", [(2, 65, RB), (2, 129, JAC), (2, 513, RB), (2, 1025, RB), (3, 17, RB),
                                            (3, 33, JAC), (3, 65, RB), (3, 129, RB)])
def test_fp16_refinement_solve_matches_oracle(dim, n, smoother, dev_ok):
    f = inputs.uniform_rhs(dim, n, 25)
    omega = 1.0 if smoother == RB else 0.8
    u_exp, h_exp, rc = oracle.solve_ir_f16(np.zeros_like(f), f, tol=1e-8, max_cycles=30, smoother=smoother,
                                           omega=omega)
    st, cyc, h, u = solve16(dim, n, f, smoother=smoother)
    assert rc == 0 and st == 0 and cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)


def test_fp16_solve_from_nonzero_guess(dev_ok):
    dim, n = 3, 33
    f = inputs.uniform_rhs(dim, n, 27)
    u0 = inputs.random_guess(dim, n, 28)
    u_exp, h_exp, _ = oracle.solve_ir_f16(u0, f, tol=1e-9, max_cycles=30)
    st, cyc, h, u = solve16(dim, n, f, tol=1e-9, u0=u0)
    assert cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)


def test_fp16_refinement_reaches_fp64_solution(dev_ok):
    """Driven to 1e-12, the binary16 form's answer agrees with the FP64 oracle to 1e-10."""
    dim, n = 3, 65
    f = inputs.uniform_rhs(dim, n, 21)
    u64, _, _ = oracle.solve(np.zeros_like(f), f, tol=1e-12, max_cycles=40)
    st, cyc, h, u = solve16(dim, n, f, tol=1e-12, max_cycles=60)
    assert st == 0 and h[-1] <= 1e-12 * h[0]
    assert np.linalg.norm(u - u64) <= 1e-10 * np.linalg.norm(u64)


def test_fp16_vcycle_entry_is_one_refinement_step(dev_ok):
    m = mg()
    dim, n = 2, 129
    f = inputs.uniform_rhs(dim, n, 41)
    u0 = inputs.random_guess(dim, n, 42)
    expect, _, _ = oracle.solve_ir_f16(u0, f, tol=0.0, max_cycles=1)
    s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP16_IR))
    ud = dev(u0)
    s.vcycle(ud, dev(f))
    assert same(host(ud), expect)
    s.close()


def test_fp16_rejects_coefficient_field(dev_ok):
    m = mg()
    n = 17
    k = dev(np.ones((n,) * 3))
    with pytest.raises(m.MGError) as ei:
        m.Solver(m.Params(dim=3, n=n, op=m.OP_VARCOEF_NODAL, k=k, precision=m.PREC_FP16_IR))
    assert ei.value.code == m.MG_ENOTSUP


def test_fp16_repeated_solves_on_one_context(dev_ok):
    """The scale state of one solve does not leak into the next."""
    m = mg()
    dim, n = 3, 33
    s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP16_IR))
    for seed, amp in [(51, 1.0), (52, 1e-6), (53, 1e5)]:
        f = inputs.uniform_rhs(dim, n, seed) * amp
        u_exp, h_exp, _ = oracle.solve_ir_f16(np.zeros_like(f), f, tol=1e-8, max_cycles=30)
        u = dev(np.zeros_like(f))
        st, cyc, h = s.solve(u, dev(f), tol=1e-8, max_cycles=30)
        assert cyc == len(h_exp) - 1
        np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
        assert same(host(u), u_exp)
    s.close()
