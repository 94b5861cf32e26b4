"""Parity of the cell-centred Neumann form (MG_BC_NEUMANN_CC) with the CPU
oracle: n = 2^L cells per axis, zero-flux boundary, averaging restriction,
constant interpolation, mean-zero projection of f and of the iterate.  The
per-cell expressions and the order of the fixed-order sums are the same on
both sides, so fields are compared bit for bit and solve histories to 1e-12
relative per cycle (the norm's partial sums are summed in another order).
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


SIZES = [(2, 2), (2, 4), (2, 64), (2, 256), (3, 2), (3, 8), (3, 32), (3, 64)]


@pytest.mark.parametrize("dim,n", SIZES)
@pytest.mark.parametrize("smoother", [RB, JAC])
def test_cc_sweep_bitwise(dim, n, smoother, dev_ok):
    u, f = inputs.random_cells(dim, n, 1), inputs.random_cells(dim, n, 2, 50.0)
    omega = 1.0 if smoother == RB else 0.8
    expect = oracle.cc_smooth(u, f, smoother, omega)
    out = dev(np.zeros_like(u))
    mg().mg_level_cc_smooth(dev(u), dev(f), out, smoother=smoother, omega=omega)
    assert np.array_equal(host(out), expect)


@pytest.mark.parametrize("dim,n", SIZES)
def test_cc_restrict_and_prolong_bitwise(dim, n, dev_ok):
    u, f = inputs.random_cells(dim, n, 3), inputs.random_cells(dim, n, 4, 50.0)
    expect = oracle.cc_restrict(oracle.cc_residual(u, f))
    fc = dev(np.zeros((n // 2,) * dim))
    mg().mg_level_cc_residual_restrict(dev(u), dev(f), fc)
    assert np.array_equal(host(fc), expect)
    ec = inputs.random_cells(dim, n // 2, 5)
    ud = dev(u)
    mg().mg_level_cc_prolong_correct(ud, dev(ec))
    assert np.array_equal(host(ud), oracle.cc_prolong_correct(u, ec))


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 512), (3, 4), (3, 128)])
def test_cc_remove_mean_bitwise(dim, n, dev_ok):
    v = inputs.random_cells(dim, n, 6) + 0.3
    mean = oracle.cc_sum(v) / v.size
    vd = dev(v)
    got = mg().mg_level_cc_remove_mean(vd)
    assert got == mean
    assert np.array_equal(host(vd), v - mean)


def cc_solve_gpu(dim, n, f, smoother=RB, cycle=0, tol=1e-10, max_cycles=60, u0=None):
    m = mg()
    s = m.Solver(m.Params(dim=dim, n=n, bc=m.BC_NEUMANN_CC, smoother=smoother, cycle=cycle))
    u = dev(np.zeros_like(f) if u0 is None else u0)
    st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
    out = host(u)
    s.close()
    return st, cyc, np.array(hist), out


@pytest.mark.parametrize("dim,n,smoother,cycle", [(2, 64, RB, 0), (2, 256, JAC, 0), (2, 1024, RB, 0), (2, 128, RB, 1),
                                                  (2, 32, JAC, 2), (3, 16, RB, 0), (3, 64, RB, 0), (3, 32, JAC, 1),
                                                  (3, 128, RB, 0), (3, 8, RB, 2), (2, 2, RB, 0)])
def test_cc_solve_matches_oracle(dim, n, smoother, cycle, dev_ok):
    f = inputs.random_cells(dim, n, 7) + 0.25  # a mean the solve projects away
    omega = 1.0 if smoother == RB else 0.8
    u_exp, h_exp, rc, _ = oracle.cc_solve(np.zeros_like(f), f, tol=1e-10, max_cycles=60, smoother=smoother,
                                          omega=omega, cycle=cycle)
    st, cyc, h, u = cc_solve_gpu(dim, n, f, smoother, cycle)
    assert cyc == len(h_exp) - 1 and st == rc
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert np.array_equal(u, u_exp)


def test_cc_solve_from_nonzero_guess_and_vcycle_entry(dev_ok):
    m = mg()
    dim, n = 3, 32
    f = inputs.random_cells(dim, n, 8)
    u0 = inputs.random_cells(dim, n, 9, 3.0)
    u_exp, h_exp, _, _ = oracle.cc_solve(u0, f, tol=1e-9, max_cycles=40)
    st, cyc, h, u = cc_solve_gpu(dim, n, f, tol=1e-9, max_cycles=40, u0=u0)
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert np.array_equal(u, u_exp)
    # one cycle of Algorithm 1 on (u0, f) as given
    s = m.Solver(m.Params(dim=dim, n=n, bc=m.BC_NEUMANN_CC))
    ud = dev(u0)
    s.vcycle(ud, dev(f))
    assert np.array_equal(host(ud), oracle.cc_cycle(u0, f))
    assert s.residual_norm(ud, dev(f)) == pytest.approx(oracle.cc_residual_norm(oracle.cc_cycle(u0, f), f), rel=1e-13)
    s.close()


def test_cc_parameters_rejected(dev_ok):
    m = mg()
    for kw, code in [(dict(n=48), m.MG_EINVAL), (dict(n=1), m.MG_EINVAL), (dict(precision=m.PREC_FP32_IR), m.MG_ENOTSUP),
                     (dict(coarse_n=9), m.MG_ENOTSUP), (dict(smoother=m.SMOOTH_RBGS_SYM), m.MG_EINVAL)]:
        args = dict(dim=2, n=64, bc=m.BC_NEUMANN_CC)
        args.update(kw)
        with pytest.raises(m.MGError) as ei:
            m.Solver(m.Params(**args))
        assert ei.value.code == code, kw
