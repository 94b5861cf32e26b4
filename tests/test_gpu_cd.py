"""Parity of the complex-diffusion form (Section 4, Eq. (2): complex
diffusivity g(Im u) = e^{i theta} / (1 + (Im u / (k theta))^2), cell-centred
Neumann grid, implicit Euler, FAS with lagged diffusivity) with the CPU
oracle.  Every per-cell complex expression is evaluated in the same order on
both sides, so operator values and FAS iterates are compared bit for bit; the
residual norms of a run to 1e-12 relative (the GPU sums per block of cells,
the oracle per x-row, plane and grid).

Inputs: the paper's denoising workload in synthetic form, a disc (2D) or ball
(3D) of value 1 on 0 plus Gaussian noise, real-valued at t = 0.
"""

import math

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


SIZES = [(2, 2), (2, 4), (2, 64), (2, 256), (3, 2), (3, 8), (3, 32), (3, 128)]  # 3D tiles from 128 cells


@pytest.mark.parametrize("dim,n", SIZES)
def test_cd_apply_bitwise(dim, n, dev_ok):
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u = inputs.random_complex(dim, n, 1)
    expect = oracle.cd_apply(u, P)
    ctx = mg().mg_cdiff_setup(dim, n, P.tau, P.theta, P.k)
    try:
        out = dev(np.zeros_like(u))
        mg().mg_cdiff_apply(ctx, dev(u), out)
        assert np.array_equal(host(out), expect)
    finally:
        mg().mg_destroy(ctx)


@pytest.mark.parametrize("dim,n", SIZES)
@pytest.mark.parametrize("smoother,nu", [(RB, (2, 2)), (RB, (1, 0)), (RB, (0, 3)), (JAC, (2, 2)), (JAC, (3, 1))])
def test_cd_fas_cycle_bitwise(dim, n, smoother, nu, dev_ok):
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 2)
    f = u0 / P.tau + 0.05 * inputs.random_complex(dim, n, 3)
    omega = 1.0 if smoother == RB else 0.8
    expect = u0
    for _ in range(2):
        expect = oracle.cd_fas(expect, f, P, smoother, omega, *nu)
    ctx = mg().mg_cdiff_setup(dim, n, P.tau, P.theta, P.k, smoother=smoother, nu1=nu[0], nu2=nu[1])
    try:
        u, fd = dev(u0), dev(f)
        mg().mg_cdiff_fas(ctx, u, fd)
        mg().mg_cdiff_fas(ctx, u, fd)
        assert np.array_equal(host(u), expect)
    finally:
        mg().mg_destroy(ctx)


@pytest.mark.parametrize("dim,n,smoother,nu", [(3, 256, RB, (2, 2)), (3, 256, JAC, (2, 2)), (2, 4096, RB, (2, 2)),
                                               (2, 4096, JAC, (2, 2)), (3, 256, RB, (1, 0)), (3, 256, JAC, (3, 1)),
                                               (2, 4096, JAC, (0, 3)), (2, 4096, RB, (1, 0))])
def test_cd_fas_cycle_bitwise_full_size(dim, n, smoother, nu, dev_ok):
    """Table 2's sizes in the launch shapes the benchmark times (3D red-black
    boxes with 16-plane chunks at 256^3 and 8 at 128^3, Jacobi chunks of 8;
    2D boxes over 4096^2): one FAS cycle bit for bit, with the correction in
    the first post-smoothing sweep (nu2 >= 1) or as its own pass (nu2 = 0)."""
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 8)
    f = u0 / P.tau + 0.05 * inputs.random_complex(dim, n, 9)
    omega = 1.0 if smoother == RB else 0.8
    expect = oracle.cd_fas(u0, f, P, smoother, omega, *nu)
    ctx = mg().mg_cdiff_setup(dim, n, P.tau, P.theta, P.k, smoother=smoother, nu1=nu[0], nu2=nu[1])
    try:
        u = dev(u0)
        mg().mg_cdiff_fas(ctx, u, dev(f))
        assert np.array_equal(host(u), expect)
    finally:
        mg().mg_destroy(ctx)


@pytest.mark.parametrize("dim,n,steps,smoother", [(3, 256, 1, RB), (2, 4096, 1, JAC)])
def test_cd_run_matches_oracle_full_size(dim, n, steps, smoother, dev_ok):
    """One implicit-Euler step at Table 2's sizes (the residual norm in the
    benchmark's launch shape): cycle count equal, the field bit for bit, the
    residual history to 1e-12 relative."""
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 5)
    omega = 1.0 if smoother == RB else 0.8
    u_exp, cyc_exp, hist_exp, rc_exp = oracle.cd_run(u0, P, steps=steps, tol=1e-5, max_cycles=12, smoother=smoother,
                                                     omega=omega)
    ctx = mg().mg_cdiff_setup(dim, n, P.tau, P.theta, P.k, smoother=smoother)
    try:
        u = dev(u0)
        st, cyc, hist = mg().mg_cdiff_run(ctx, u, steps, 1e-5, 12)
        assert (st == 0) == (rc_exp == 0)
        assert list(cyc) == list(cyc_exp)
        for h, he in zip(hist, hist_exp):
            np.testing.assert_allclose(h, he, rtol=1e-12, atol=0)
        assert np.array_equal(host(u), u_exp)
    finally:
        mg().mg_destroy(ctx)


@pytest.mark.parametrize("dim,n,steps", [(2, 128, 3), (2, 512, 2), (3, 32, 3), (3, 64, 2), (3, 128, 1)])
@pytest.mark.parametrize("smoother", [RB, JAC])
def test_cd_run_matches_oracle(dim, n, steps, smoother, dev_ok):
    """Implicit-Euler steps with FAS per step: cycle counts equal, the final
    field bit for bit, the residual histories to 1e-12 relative."""
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 5)
    omega = 1.0 if smoother == RB else 0.8
    tol, mc = 1e-5, 12
    u_exp, cyc_exp, hist_exp, rc_exp = oracle.cd_run(u0, P, steps=steps, tol=tol, max_cycles=mc, smoother=smoother,
                                                     omega=omega)
    ctx = mg().mg_cdiff_setup(dim, n, P.tau, P.theta, P.k, smoother=smoother)
    try:
        u = dev(u0)
        st, cyc, hist = mg().mg_cdiff_run(ctx, u, steps, tol, mc)
        assert (st == 0) == (rc_exp == 0)
        assert list(cyc) == list(cyc_exp)
        for h, he in zip(hist, hist_exp):
            np.testing.assert_allclose(h, he, rtol=1e-12, atol=0)
        assert np.array_equal(host(u), u_exp)
    finally:
        mg().mg_destroy(ctx)


def test_cd_run_reduces_residual_by_1e5_within_five_cycles(dev_ok):
    """Section 4's complex-diffusion statement at 1024^2 cells: every step
    reaches a 1e5 residual reduction within five V(2,2) cycles, and the field
    keeps its complex mass (zero flux through the boundary) up to tau times
    the remaining residual's sum."""
    n = 1024
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(2, n, 7)
    ctx = mg().mg_cdiff_setup(2, n, P.tau, P.theta, P.k)
    try:
        u = dev(u0)
        st, cyc, hist = mg().mg_cdiff_run(ctx, u, 3, 1e-5, 5)
        assert st == 0 and all(1 <= c <= 5 for c in cyc)
        u1 = host(u)
        assert abs(u1.sum() - u0.sum()) <= 1e-6 * np.abs(u0).sum()
        assert np.abs(u1.imag).max() > 1e-5
    finally:
        mg().mg_destroy(ctx)


def test_cd_rejects_bad_arguments(dev_ok):
    import torch

    m = mg()
    for kw in [dict(dim=4, n=8), dict(dim=2, n=6), dict(dim=2, n=8192), dict(dim=3, n=512)]:
        with pytest.raises(m.MGError):
            m.mg_cdiff_setup(kw["dim"], kw["n"], 1e-3)
    for bad in [dict(tau=0.0), dict(theta=0.0), dict(theta=math.pi / 2), dict(k=-1.0), dict(smoother=2),
                dict(nu1=17)]:
        args = dict(tau=1e-3, theta=math.pi / 30, k=0.1)
        args.update(bad)
        with pytest.raises(m.MGError):
            m.mg_cdiff_setup(2, 8, **args)
    ctx = m.mg_cdiff_setup(2, 8, 1e-3)
    try:
        buf = torch.zeros(2 * 64 + 1, dtype=torch.float64, device="cuda")
        with pytest.raises(m.MGError):  # 8-byte aligned complex array
            m._check(m.lib().mg_cdiff_apply(ctx, buf.data_ptr() + 8, buf.data_ptr()), "mg_cdiff_apply")
        u = dev(np.zeros((8, 8), np.complex128))
        with pytest.raises(m.MGError):  # a Poisson call on a complex-diffusion handle
            m._check(m.lib().mg_vcycle(ctx, u.data_ptr(), u.data_ptr()), "mg_vcycle")
        assert m.mg_num_levels(ctx) == 4
    finally:
        m.mg_destroy(ctx)
