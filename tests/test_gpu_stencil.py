"""Parity of the constant-stencil operator (MG_OP_CONST_STENCIL; Section 2.2's
stencil with constant entries, re-discretised with each level's h) with the
CPU oracle.  Per-node expressions are the same on both sides, so fields are
compared bit for bit and solve histories to max(1e-12, (N-1) 2^-53) relative
per cycle (the GPU norm sums per block of nodes, the oracle per plane).
"""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

RB, JAC, SYM = 0, 1, 2
V, W, F = 0, 1, 2

SKEW2 = [4.4, -1.3, -0.7, -1.1, -0.9]
SKEW3 = [6.5, -1.2, -0.8, -1.15, -0.85, -1.3, -0.7]
ZSUM2 = [3.2, -1.0, -1.0, -0.6, -0.6]
ZSUM3 = [4.2, -1.0, -1.0, -0.7, -0.7, -0.4, -0.4]
ZSKEW3 = [6.0, -1.2, -0.8, -1.1, -0.9, -1.05, -0.95]


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


def arrays(dim, n, seed):
    u = inputs.random_guess(dim, n, 40 + seed)
    f = inputs.uniform_rhs(dim, n, 50 + seed) * 50.0
    return u, f


SIZES = [(2, 5), (2, 33), (2, 129), (2, 257), (3, 5), (3, 17), (3, 65)]


def sten(dim, kind):
    return {("skew", 2): SKEW2, ("skew", 3): SKEW3, ("zsum", 2): ZSUM2, ("zsum", 3): ZSUM3}[(kind, dim)]


@pytest.mark.parametrize("dim,n", SIZES)
@pytest.mark.parametrize("smoother", [RB, JAC, SYM])
@pytest.mark.parametrize("kind", ["skew", "zsum"])
def test_st_sweep_bitwise(dim, n, smoother, kind, dev_ok):
    st = sten(dim, kind)
    u, f = arrays(dim, n, 1)
    omega = 0.8 if smoother == JAC else 1.0
    expect = oracle.st_smooth(u, f, st, smoother, omega)
    out = dev(np.zeros_like(u))
    mg().mg_level_st_smooth(dev(u), dev(f), out, st, smoother=smoother, omega=omega)
    assert np.array_equal(host(out), expect)


@pytest.mark.parametrize("dim,n", [s for s in SIZES if s[1] >= 5])
@pytest.mark.parametrize("kind", ["skew", "zsum"])
def test_st_restrict_bitwise(dim, n, kind, dev_ok):
    st = sten(dim, kind)
    u, f = arrays(dim, n, 2)
    expect = oracle.restrict(oracle.st_residual(u, f, st))
    nc = (n - 1) // 2 + 1
    fc = dev(np.zeros((nc,) * dim))
    mg().mg_level_st_residual_restrict(dev(u), dev(f), fc, st)
    assert np.array_equal(host(fc), expect)


@pytest.mark.parametrize("dim", [2, 3])
def test_st_coarsest_bitwise(dim, dev_ok):
    st = sten(dim, "skew")
    f = np.zeros((3,) * dim)
    f[(1,) * dim] = 1.75
    u = dev(np.zeros_like(f))
    mg().mg_level_st_coarsest(u, dev(f), st)
    assert np.array_equal(host(u), oracle.st_coarsest(f, st))


def norm_rtol(dim, n):
    """The two norms sum the same N = (n-2)^dim non-negative squares in
    different orders (the oracle one plane at a time, the GPU per block of
    nodes); each sum is within (N-1) 2^-53 of the exact one relative to it,
    and the square root halves the difference."""
    return max(1e-12, ((n - 2) ** dim - 1) * 2.0**-53)


def solve_both(dim, n, st, smoother, cycle, tol=1e-10, max_cycles=30, u0=None, seed=3):
    m = mg()
    f = inputs.uniform_rhs(dim, n, seed)
    u0 = np.zeros_like(f) if u0 is None else u0
    omega = 0.8 if smoother == JAC else 1.0
    ue, he, rce = oracle.st_solve(u0, f, st, tol=tol, max_cycles=max_cycles, smoother=smoother, omega=omega,
                                  cycle=cycle)
    s = m.Solver(m.Params(dim=dim, n=n, op=m.OP_CONST_STENCIL, stencil=st, smoother=smoother, cycle=cycle))
    try:
        u = dev(u0)
        status, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
        return (ue, he, rce), (host(u), np.array(hist), status, cyc)
    finally:
        s.close()


@pytest.mark.parametrize("dim,n,st", [(2, 129, ZSUM2), (2, 513, ZSUM2), (3, 17, ZSKEW3), (3, 33, ZSUM3),
                                      (3, 65, ZSUM3)])
@pytest.mark.parametrize("smoother,cycle", [(RB, V), (JAC, V), (SYM, V), (RB, W), (RB, F)])
def test_st_solve_matches_oracle(dim, n, st, smoother, cycle, dev_ok):
    (ue, he, rce), (u, h, status, cyc) = solve_both(dim, n, st, smoother, cycle)
    assert status == rce and cyc == len(he) - 1
    np.testing.assert_allclose(h, he, rtol=norm_rtol(dim, n), atol=0)
    assert np.array_equal(u, ue)


def test_st_solve_from_nonzero_guess_and_vcycle_entry(dev_ok):
    m = mg()
    dim, n = 2, 65
    u0 = inputs.zero_boundary(inputs.random_guess(dim, n, 9))
    (ue, he, _), (u, h, _, _) = solve_both(dim, n, ZSUM2, RB, V, u0=u0, max_cycles=8, tol=0.0)
    np.testing.assert_allclose(h, he, rtol=1e-12, atol=0)
    assert np.array_equal(u, ue)
    # single cycles through mg_vcycle, and the residual norm entry
    f = inputs.uniform_rhs(dim, n, 3)
    expect = oracle.st_solve(u0, f, ZSUM2, tol=0.0, max_cycles=2)[0]
    s = m.Solver(m.Params(dim=dim, n=n, op=m.OP_CONST_STENCIL, stencil=ZSUM2))
    try:
        ud, fd = dev(u0), dev(f)
        s.vcycle(ud, fd)
        s.vcycle(ud, fd)
        assert np.array_equal(host(ud), expect)
        rn = s.residual_norm(ud, fd)
        assert rn == pytest.approx(oracle.st_residual_norm(expect, f, ZSUM2), rel=1e-13)
    finally:
        s.close()


@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33)])
@pytest.mark.parametrize("smoother", [RB, JAC, SYM])
def test_laplacian_stencil_equals_laplacian_path(dim, n, smoother, dev_ok):
    """The Laplacian's stencil through the stencil kernels gives the tuned
    Laplacian path's iterates bit for bit (both equal the oracle's)."""
    m = mg()
    lap = [2.0 * dim] + [-1.0] * (2 * dim)
    f = inputs.uniform_rhs(dim, n, 4)
    out = []
    for op, st in ((m.OP_CONST_STENCIL, lap), (m.OP_LAPLACE, None)):
        s = m.Solver(m.Params(dim=dim, n=n, op=op, stencil=st, smoother=smoother))
        try:
            u = dev(np.zeros_like(f))
            status, cyc, hist = s.solve(u, dev(f), tol=1e-9, max_cycles=20)
            out.append((host(u), np.array(hist), cyc))
        finally:
            s.close()
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0])
    np.testing.assert_allclose(out[0][1], out[1][1], rtol=1e-12, atol=0)


def test_st_and_h_parameter_errors(dev_ok):
    m = mg()
    bad_inval = [dict(stencil=None), dict(stencil=[0.0, -1, -1, -1, -1]), dict(stencil=[float("nan"), -1, -1, -1, -1]),
                 dict(stencil=[4, -1, -1, float("inf"), -1]), dict(stencil=ZSUM2, h=-0.1)]
    for kw in bad_inval:
        with pytest.raises(m.MGError) as ei:
            m.mg_setup(m.Params(dim=2, n=33, op=m.OP_CONST_STENCIL, **kw))
        assert ei.value.code == m.MG_EINVAL, kw
    bad_sup = [dict(precision=m.PREC_FP32_IR), dict(precision=m.PREC_FP16_IR), dict(coarse_n=5), dict(h=0.5)]
    for kw in bad_sup:
        with pytest.raises(m.MGError) as ei:
            m.mg_setup(m.Params(dim=2, n=33, op=m.OP_CONST_STENCIL, stencil=ZSUM2, **kw))
        assert ei.value.code == m.MG_ENOTSUP, kw
    # h: the unit domain's spacing is accepted on every path, any other is not built
    for op, st in ((m.OP_CONST_STENCIL, ZSUM2), (m.OP_LAPLACE, None)):
        ctx = m.mg_setup(m.Params(dim=2, n=33, op=op, stencil=st, h=1.0 / 32))
        m.mg_destroy(ctx)
        with pytest.raises(m.MGError) as ei:
            m.mg_setup(m.Params(dim=2, n=33, op=op, stencil=st, h=1.0 / 33))
        assert ei.value.code == m.MG_ENOTSUP
    ctx = m.mg_setup(m.Params(dim=2, n=32, bc=m.BC_NEUMANN_CC, h=1.0 / 32))
    m.mg_destroy(ctx)
    with pytest.raises(m.MGError):
        m.mg_setup(m.Params(dim=2, n=32, bc=m.BC_NEUMANN_CC, h=1.0 / 31))
    # batches take the Laplacian only
    with pytest.raises(m.MGError) as ei:
        m.mg_batch_setup([m.Params(dim=2, n=33, op=m.OP_CONST_STENCIL, stencil=ZSUM2, precision=m.PREC_FP32_IR)])
    assert ei.value.code in (m.MG_ENOTSUP, m.MG_EINVAL)
    # no tuned tiles on a stencil context
    ctx = m.mg_setup(m.Params(dim=2, n=33, op=m.OP_CONST_STENCIL, stencil=ZSUM2))
    try:
        assert m.mg_num_levels(ctx) == 5
        with pytest.raises(m.MGError):
            m.mg_tile_config(ctx, 0, 0)
    finally:
        m.mg_destroy(ctx)
