"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Per-point arithmetic is the same expression on both sides and neither side
contracts to FMA, so every field the HIP kernels produce is compared bit for
bit with the oracle's (torch.equal / numpy.array_equal).  Residual norms are
sums in different orders and are compared to 1e-13 relative; solve histories
to 1e-12 relative per cycle.  Sizes span several tiles with ragged last tiles
(3D tiles are 60 x 12 nodes by default, 2D 60 x 28), and tile shapes are varied.
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
    return a.shape == b.shape and np.array_equal(a, b)


def over_row_limit(dim, by, dt, varcoef, waves=0):
    """3D sweeps hold by / waves rows per thread (4 wavefronts unless given): at
    most 2 in FP64 with a coefficient field, 4 in FP64 or with one, 8
    otherwise; with one wavefront per tile (waves = 1) the tile has 12 rows at
    most in FP32 without coefficients, 8 in FP32 with them or FP64 without,
    none in FP64 with them.  The library rejects more (they would not fit the
    register file)."""
    if dim != 3 or not by:
        return False
    fp64 = dt == np.float64
    if waves == 1:
        return by > (0 if (fp64 and varcoef) else (8 if (fp64 or varcoef) else 12))
    return by // (waves or 4) > (2 if (fp64 and varcoef) else (4 if (fp64 or varcoef) else 8))


def case_arrays(dim, n, dt, varcoef, seed=0):
    u = inputs.random_guess(dim, n, 100 + seed).astype(dt)
    f = (inputs.uniform_rhs(dim, n, 200 + seed) * 50.0).astype(dt)
    k = inputs.varcoef_k(n, 300 + seed, dim=dim).astype(dt) if varcoef else None
    return u, f, k


SMOOTH_CASES = [
    # dim, n, by, zchunk, prefetch, waves (0: library default); 3D boxes are 128 nodes wide
    (2, 5, 0, 0, 0, 0), (2, 9, 8, 0, 0, 0), (2, 33, 16, 0, 0, 0), (2, 129, 0, 0, 0, 0), (2, 257, 32, 0, 0, 0),
    (2, 65, 8, 0, 0, 0), (3, 5, 0, 0, 1, 0), (3, 9, 8, 1, 2, 0), (3, 17, 16, 3, 1, 8), (3, 17, 16, 3, 1, 0),
    (3, 33, 0, 0, 2, 0), (3, 65, 32, 7, 2, 8), (3, 65, 8, 64, 1, 0), (3, 129, 16, 128, 2, 8), (3, 33, 32, 2, 1, 0),
    (3, 33, 16, 5, 2, 4), (3, 129, 32, 16, 1, 8), (3, 257, 16, 40, 1, 8),
    (3, 65, 8, 7, 1, 1), (3, 129, 12, 16, 2, 1), (3, 33, 12, 5, 1, 1), (3, 17, 8, 0, 2, 1),
]


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", SMOOTH_CASES)
@pytest.mark.parametrize("smoother", [RB, JAC])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("varcoef", [False, True])
def test_smooth_sweep_bitwise(dim, n, by, zc, pd, wv, smoother, dt, varcoef, dev_ok):
    u, f, k = case_arrays(dim, n, dt, varcoef, seed=n)
    omega = 1.0 if smoother == RB else 0.8
    expect = oracle.smooth(u, f, smoother=smoother, omega=omega, k=k)
    ud, fd = dev(u), dev(f)
    out = dev(np.zeros_like(u))
    kd = dev(k) if k is not None else None
    if over_row_limit(dim, by, dt, varcoef, wv):
        with pytest.raises(mg().MGError) as ei:
            mg().mg_level_smooth(ud, fd, out, smoother=smoother, omega=omega, k=kd, by=by, zchunk=zc, prefetch=pd,
                                 waves=wv)
        assert ei.value.code == mg().MG_EINVAL
        return
    mg().mg_level_smooth(ud, fd, out, smoother=smoother, omega=omega, k=kd, by=by, zchunk=zc, prefetch=pd, waves=wv)
    assert same(host(out), expect)
    # the other block-to-tile order: the same sweep, bit for bit
    out2 = dev(np.zeros_like(u))
    mg().mg_level_smooth(ud, fd, out2, smoother=smoother, omega=omega, k=kd, by=by, zchunk=zc, prefetch=pd, waves=wv,
                         order=1)
    assert same(host(out2), expect)


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", [(2, 65, 16, 0, 0, 0), (3, 33, 16, 5, 1, 8), (3, 17, 8, 0, 2, 0),
                                              (3, 65, 32, 9, 2, 8), (3, 129, 16, 11, 1, 4), (3, 65, 12, 9, 1, 1),
                                              (3, 33, 8, 3, 2, 1), (3, 129, 8, 7, 1, 1), (3, 9, 12, 2, 2, 1),
                                              (3, 257, 8, 33, 1, 1)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_smooth_zero_guess_bitwise(dim, n, by, zc, pd, wv, dt, dev_ok):
    """wv = 1 (3D): one wavefront per tile, rows in registers (several x
    tiles with a ragged last one at n = 129 and 257)."""
    _, f, _ = case_arrays(dim, n, dt, False, seed=3)
    expect = oracle.smooth(np.zeros_like(f), f)
    out = dev(np.zeros_like(f))
    if over_row_limit(dim, by, dt, False, wv):
        with pytest.raises(mg().MGError):
            mg().mg_level_smooth(None, dev(f), out, zero_guess=True, by=by, zchunk=zc, prefetch=pd, waves=wv)
        return
    mg().mg_level_smooth(None, dev(f), out, zero_guess=True, by=by, zchunk=zc, prefetch=pd, waves=wv)
    assert same(host(out), expect)


FUSED_CASES = [(2, 9, 0, 0, 0, 0), (2, 65, 0, 0, 0, 0), (2, 257, 0, 0, 0, 0), (2, 5, 8, 0, 0, 0),
               (2, 129, 8, 0, 0, 0), (2, 129, 32, 0, 0, 0), (2, 513, 16, 0, 0, 0),
               (3, 5, 0, 0, 0, 0), (3, 9, 8, 1, 1, 0), (3, 17, 16, 3, 2, 8), (3, 33, 8, 5, 1, 0),
               (3, 33, 32, 2, 2, 8), (3, 65, 16, 7, 1, 8), (3, 65, 0, 0, 0, 0), (3, 129, 16, 13, 1, 8),
               (3, 33, 16, 5, 2, 4), (3, 129, 32, 7, 1, 8), (3, 65, 8, 7, 2, 1), (3, 129, 12, 13, 1, 1),
               (3, 33, 8, 5, 1, 1)]


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", FUSED_CASES)
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("smoother", [RB, JAC])
@pytest.mark.parametrize("varcoef", [False, True])
def test_smooth_with_fused_correction_bitwise(dim, n, by, zc, pd, wv, dt, smoother, varcoef, dev_ok):
    """First post-smoothing sweep with the coarse-grid correction added while
    loading: equals interpolation + correction followed by the sweep.  Odd
    z-chunks put the first plane of a chunk on both parities."""
    u, f, k = case_arrays(dim, n, dt, varcoef, seed=5)
    nc = (n - 1) // 2 + 1
    ec = inputs.random_guess(dim, nc, 77).astype(dt)
    omega = 1.0 if smoother == RB else 0.8
    expect = oracle.smooth(oracle.prolong_correct(u, ec), f, smoother=smoother, omega=omega, k=k)
    out = dev(np.zeros_like(u))
    kd = dev(k) if varcoef else None
    if over_row_limit(dim, by, dt, varcoef, wv):
        with pytest.raises(mg().MGError) as ei:
            mg().mg_level_smooth(dev(u), dev(f), out, smoother=smoother, omega=omega, k=kd, ec=dev(ec), by=by,
                                 zchunk=zc, prefetch=pd, waves=wv)
        assert ei.value.code == mg().MG_EINVAL
        return
    mg().mg_level_smooth(dev(u), dev(f), out, smoother=smoother, omega=omega, k=kd, ec=dev(ec), by=by, zchunk=zc,
                         prefetch=pd, waves=wv)
    assert same(host(out), expect)


@pytest.mark.parametrize("dim,n,by,zc", [(2, 5, 0, 0), (2, 65, 8, 0), (2, 129, 32, 0), (2, 257, 16, 0),
                                         (3, 5, 0, 0), (3, 17, 8, 1), (3, 33, 16, 2), (3, 65, 0, 0),
                                         (3, 129, 32, 9)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("varcoef", [False, True])
def test_residual_restrict_bitwise(dim, n, by, zc, dt, varcoef, dev_ok):
    u, f, k = case_arrays(dim, n, dt, varcoef, seed=7)
    expect = oracle.restrict(oracle.residual(u, f, k=k))
    nc = (n - 1) // 2 + 1
    fc = dev(np.zeros((nc,) * dim, dtype=dt))
    mg().mg_level_residual_restrict(dev(u), dev(f), fc, k=dev(k) if k is not None else None, by=by, zchunk=zc)
    assert same(host(fc), expect)


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 129), (3, 5), (3, 33), (3, 65)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_prolong_correct_bitwise(dim, n, dt, dev_ok):
    u, _, _ = case_arrays(dim, n, dt, False, seed=9)
    nc = (n - 1) // 2 + 1
    ec = inputs.random_guess(dim, nc, 99).astype(dt)
    expect = oracle.prolong_correct(u, ec)
    ud = dev(u)
    mg().mg_level_prolong_correct(ud, dev(ec))
    assert same(host(ud), expect)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("varcoef", [False, True])
def test_coarsest_bitwise(dim, varcoef, dev_ok):
    f = np.zeros((3,) * dim)
    f[(1,) * dim] = 0.37
    k = inputs.varcoef_k(3, 4, dim=dim) if varcoef else None
    expect = oracle.coarsest(np.zeros_like(f), f, k=k)
    ud = dev(np.zeros_like(f))
    mg().mg_level_coarsest(ud, dev(f), k=dev(k) if k is not None else None)
    assert same(host(ud), expect)


@pytest.mark.parametrize("dim,n,by,zc,pd,wv,pr", [(2, 65, 0, 0, 0, 0, 0), (2, 257, 8, 0, 0, 0, 0),
                                                 (3, 33, 0, 0, 0, 0, 0), (3, 65, 16, 3, 1, 0, 0),
                                                 (3, 65, 8, 7, 2, 4, 0), (3, 65, 16, 5, 1, 8, 0),
                                                 (3, 129, 32, 16, 2, 8, 0), (3, 33, 32, 7, 2, 8, 0),
                                                 (3, 33, 16, 1, 2, 4, 0), (3, 5, 8, 1, 1, 4, 1), (3, 33, 8, 4, 1, 4, 1),
                                                 (3, 129, 8, 16, 2, 4, 1), (3, 257, 16, 9, 1, 8, 1),
                                                 (3, 65, 32, 5, 2, 8, 1), (3, 257, 16, 31, 2, 4, 1),
                                                 (3, 9, 16, 2, 2, 4, 1), (2, 65, 16, 8, 1, 4, 1),
                                                 (2, 257, 16, 32, 2, 4, 1), (2, 129, 16, 5, 1, 4, 1),
                                                 (2, 5, 16, 1, 2, 4, 1), (2, 1025, 16, 100, 2, 4, 1),
                                                 (2, 513, 0, 0, 0, 0, 1)])
@pytest.mark.parametrize("varcoef", [False, True])
def test_refinement_pass(dim, n, by, zc, pd, wv, pr, varcoef, dev_ok):
    """pr: two nodes per lane (128 computed nodes per tile row, 16-byte pair
    accesses, the two x-neighbours outside the tile loaded on their own);
    Laplacian only.  In 2D each wavefront marches zc rows along y."""
    import torch

    u, f, k = case_arrays(dim, n, np.float64, varcoef, seed=11)
    e = (inputs.random_guess(dim, n, 12) * 1e-3).astype(np.float32)
    uo = dev(np.zeros_like(u))
    r = torch.zeros(u.shape, dtype=torch.float32, device="cuda")
    if pr and varcoef:
        with pytest.raises(mg().MGError) as ei:
            mg().mg_level_ir_update(dev(u), dev(e), dev(f), uo, r, k=dev(k), by=by, zchunk=zc, prefetch=pd,
                                    waves=wv, pairs=pr)
        assert ei.value.code == mg().MG_EINVAL
        return
    u_exp, r_exp, rho_exp = oracle.ir_update(u, e, f, k=k)
    rho = mg().mg_level_ir_update(dev(u), dev(e), dev(f), uo, r, k=dev(k) if k is not None else None, by=by,
                                  zchunk=zc, prefetch=pd, waves=wv, pairs=pr)
    assert same(host(uo), u_exp)
    assert same(host(r), r_exp)
    assert rho == pytest.approx(rho_exp, rel=1e-13)


def test_refinement_pass_pairs_row_limit(dev_ok):
    """Two nodes per lane hold at most four rows per thread (32 rows need
    eight wavefronts): other shapes are rejected before any launch."""
    import torch

    u, f, _ = case_arrays(3, 33, np.float64, False, seed=11)
    e = np.zeros(u.shape, np.float32)
    uo = dev(np.zeros_like(u))
    r = torch.zeros(u.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(mg().MGError) as ei:
        mg().mg_level_ir_update(dev(u), dev(e), dev(f), uo, r, by=32, zchunk=4, prefetch=1, waves=4, pairs=1)
    assert ei.value.code == mg().MG_EINVAL


# ---------------------------------------------------------------- full solves
def run_solve(dim, n, f, k=None, smoother=RB, precision=0, tol=0.0, max_cycles=10, u0=None):
    m = mg()
    p = m.Params(dim=dim, n=n, smoother=smoother, precision=precision,
                 op=m.OP_VARCOEF_NODAL if k is not None else m.OP_LAPLACE,
                 k=dev(k) if k is not None else None)
    s = m.Solver(p)
    u = dev(np.zeros_like(f) if u0 is None else u0)
    st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
    out = host(u)
    s.close()
    return st, cyc, np.array(hist), out


@pytest.mark.parametrize("smoother", [RB, JAC])
def test_poisson2d_129_sine_history_and_field(smoother, dev_ok):
    """The 129 x 129 workload: ten V(2,2) cycles, FP64."""
    f = inputs.sine_rhs(2, 129)
    omega = 1.0 if smoother == RB else 0.8
    u_exp, h_exp, _ = oracle.solve(np.zeros_like(f), f, tol=0.0, max_cycles=10, smoother=smoother, omega=omega)
    st, cyc, h, u = run_solve(2, 129, f, smoother=smoother)
    assert cyc == 10
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)


@pytest.mark.parametrize("dim,n,varcoef,smoother", [(3, 65, False, RB), (3, 33, True, RB), (3, 33, False, JAC),
                                                    (2, 257, True, RB), (2, 1025, False, RB), (3, 129, False, RB)])
def test_fp64_solve_matches_oracle(dim, n, varcoef, smoother, dev_ok):
    f = inputs.uniform_rhs(dim, n, 5)
    k = inputs.varcoef_k(n, 6, dim=dim) if varcoef else None
    omega = 1.0 if smoother == RB else 0.8
    u_exp, h_exp, rc = oracle.solve(np.zeros_like(f), f, tol=1e-10, max_cycles=30, smoother=smoother, omega=omega,
                                    k=k)
    st, cyc, h, u = run_solve(dim, n, f, k=k, smoother=smoother, tol=1e-10, max_cycles=30)
    assert cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)
    assert st == 0


@pytest.mark.parametrize("dim,n,varcoef", [(2, 129, False), (3, 65, False), (3, 33, True), (2, 513, False)])
def test_fp32_refinement_solve_matches_oracle(dim, n, varcoef, dev_ok):
    f = inputs.uniform_rhs(dim, n, 15)
    k = inputs.varcoef_k(n, 16, dim=dim) if varcoef else None
    u_exp, h_exp, rc = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=30, k=k)
    st, cyc, h, u = run_solve(dim, n, f, k=k, precision=1, tol=1e-8, max_cycles=30)
    assert st == 0 and cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)


def test_fp32_refinement_reaches_fp64_solution(dev_ok):
    """Mixed precision driven to 1e-12: the answer agrees with the FP64 oracle to 1e-10."""
    dim, n = 3, 65
    f = inputs.uniform_rhs(dim, n, 21)
    u64, h64, _ = oracle.solve(np.zeros_like(f), f, tol=1e-12, max_cycles=40)
    st, cyc, h, u = run_solve(dim, n, f, precision=1, tol=1e-12, max_cycles=40)
    assert h[-1] <= 1e-12 * h[0]
    assert np.linalg.norm(u - u64) <= 1e-10 * np.linalg.norm(u64)


def test_vcycle_entry_and_residual_norm(dev_ok):
    m = mg()
    dim, n = 3, 33
    f = inputs.uniform_rhs(dim, n, 31)
    u0 = inputs.random_guess(dim, n, 32)
    expect = oracle.vcycle(u0, f)
    s = m.Solver(m.Params(dim=dim, n=n))
    ud, fd = dev(u0), dev(f)
    s.vcycle(ud, fd)
    assert same(host(ud), expect)
    assert s.residual_norm(ud, fd) == pytest.approx(oracle.residual_norm(expect, f), rel=1e-13)
    s.close()


def test_fp32_vcycle_entry_is_one_refinement_step(dev_ok):
    m = mg()
    dim, n = 2, 129
    f = inputs.uniform_rhs(dim, n, 41)
    u0 = inputs.random_guess(dim, n, 42)
    _, r32, _ = oracle.ir_update(u0, np.zeros(f.shape, np.float32), f)
    e = oracle.vcycle(np.zeros(f.shape, np.float32), r32)
    expect, _, _ = oracle.ir_update(u0, e, f)
    s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR))
    ud = dev(u0)
    s.vcycle(ud, dev(f))
    assert same(host(ud), expect)
    s.close()


def test_setup_rejects_bad_arguments(dev_ok):
    m = mg()
    for kw in [dict(dim=2, n=128), dict(dim=4, n=9), dict(dim=2, n=9, nu1=-1), dict(dim=3, n=9, smoother=5),
               dict(dim=2, n=9, op=m.OP_VARCOEF_NODAL)]:
        with pytest.raises(m.MGError) as ei:
            m.mg_setup(m.Params(**kw))
        assert ei.value.code == m.MG_EINVAL
    with pytest.raises(m.MGError) as ei:  # no such boundary condition
        m.mg_setup(m.Params(dim=2, n=9, bc=7))
    assert ei.value.code == m.MG_ENOTSUP
    with pytest.raises(m.MGError) as ei:  # a cell-centred grid has 2^L cells per axis
        m.mg_setup(m.Params(dim=2, n=9, bc=m.BC_NEUMANN_CC))
    assert ei.value.code == m.MG_EINVAL


def test_nan_rhs_reports_divergence(dev_ok):
    f = inputs.uniform_rhs(2, 65, 1)
    f[10, 10] = np.nan
    st, cyc, h, u = run_solve(2, 65, f, tol=1e-8, max_cycles=10)
    assert st == mg().MG_EDIVERGED


def test_max_cycles_exhaustion_reports_not_converged(dev_ok):
    f = inputs.uniform_rhs(3, 33, 2)
    st, cyc, h, u = run_solve(3, 33, f, tol=1e-30, max_cycles=3)
    assert st == mg().MG_ENOTCONV and cyc == 3 and len(h) == 4


@pytest.mark.parametrize("precision", [0, 1])
def test_repeated_solves_on_one_context_are_identical(precision, dev_ok):
    """A context is reusable: back-to-back solves (same or new buffers) give the oracle's answer each time."""
    import torch

    m = mg()
    dim, n = 3, 33
    f = inputs.uniform_rhs(dim, n, 51)
    solve = oracle.solve if precision == 0 else oracle.solve_ir_f32
    u_exp, h_exp, _ = solve(np.zeros_like(f), f, tol=1e-8, max_cycles=30)
    s = m.Solver(m.Params(dim=dim, n=n, precision=precision))
    fd = dev(f)
    bufs = [torch.zeros(f.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    for u in [bufs[0], bufs[1], bufs[1], bufs[2], bufs[0]]:
        u.zero_()
        st, cyc, hist = s.solve(u, fd, tol=1e-8, max_cycles=30)
        assert st == 0 and cyc == len(h_exp) - 1
        np.testing.assert_allclose(hist, h_exp, rtol=1e-12, atol=0)
        assert same(host(u), u_exp)
    s.close()


@pytest.mark.parametrize("dim,n,precision", [(3, 129, 1), (3, 65, 0), (2, 1025, 1)])
def test_solve_independent_of_launch_geometry(dim, n, precision, dev_ok, monkeypatch):
    """Autotuned tile shapes and the built-in heuristic give bit-identical solves."""
    f = inputs.uniform_rhs(dim, n, 61)
    monkeypatch.setenv("MG_AUTOTUNE", "0")
    st0, c0, h0, u0 = run_solve(dim, n, f, precision=precision, tol=1e-8, max_cycles=30)
    monkeypatch.setenv("MG_AUTOTUNE", "1")
    st1, c1, h1, u1 = run_solve(dim, n, f, precision=precision, tol=1e-8, max_cycles=30)
    assert st0 == st1 == 0 and c0 == c1
    assert same(u0, u1)
    np.testing.assert_allclose(h0, h1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("dim,n,precision,varcoef,smoother", [(2, 129, 1, False, RB), (2, 65, 1, False, RB),
                                                              (2, 257, 0, True, RB), (3, 65, 1, False, RB),
                                                              (3, 33, 0, True, JAC), (3, 17, 1, False, JAC),
                                                              (2, 33, 0, False, JAC), (3, 129, 0, False, RB)])
def test_coarse_tail_kernel_equals_level_by_level(dim, n, precision, varcoef, smoother, dev_ok, monkeypatch):
    """The coarse levels run by the single-workgroup tail kernel give the same
    bits as running them level by level (and both equal the oracle)."""
    f = inputs.uniform_rhs(dim, n, 63)
    k = inputs.varcoef_k(n, 64, dim=dim) if varcoef else None
    monkeypatch.setenv("MG_NO_TAIL", "1")
    st0, c0, h0, u0 = run_solve(dim, n, f, k=k, smoother=smoother, precision=precision, tol=1e-9, max_cycles=30)
    monkeypatch.delenv("MG_NO_TAIL")
    st1, c1, h1, u1 = run_solve(dim, n, f, k=k, smoother=smoother, precision=precision, tol=1e-9, max_cycles=30)
    assert st0 == st1 == 0 and c0 == c1
    assert same(u0, u1)
    np.testing.assert_allclose(h0, h1, rtol=1e-13, atol=0)
    omega = 1.0 if smoother == RB else 0.8
    if precision == 0:
        u_exp, _, _ = oracle.solve(np.zeros_like(f), f, tol=1e-9, max_cycles=30, smoother=smoother, omega=omega, k=k)
    else:
        u_exp, _, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-9, max_cycles=30, smoother=smoother,
                                          omega=omega, k=k)
    assert same(u1, u_exp)
