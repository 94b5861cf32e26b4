"""FP64 solves whose residual norms (Section 2.4's L2 residual of each
cycle's result, Algorithm 1's stop test) are summed by the next cycle's first
pre-smoothing sweep instead of a pass of their own: parity with the CPU oracle
and with the separate norm pass (MG_NO_FUSED_NORM=1).

The sweep writes the ping-pong partner of u, so when the stop test ends the
solve u still holds the last cycle's result: fields are compared bit for bit.
Norms sum the same squares in a different order (per workgroup of the sweep,
then the workgroups in order; the oracle per plane), so histories are compared
to max(1e-12, (N-1) 2^-53) relative, N the number of inner nodes.
"""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

RB, JAC, SYM = 0, 1, 2
V, W, F = 0, 1, 2


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


def norm_rtol(dim, n):
    return max(1e-12, ((n - 2) ** dim - 1) * 2.0**-53)


def gpu_solve(dim, n, f, u0, k=None, smoother=RB, cycle=V, nu1=2, nu2=2, tol=1e-10, max_cycles=30):
    m = mg()
    p = m.Params(dim=dim, n=n, smoother=smoother, cycle=cycle, nu1=nu1, nu2=nu2, precision=m.PREC_FP64,
                 omega=0.8 if smoother == JAC else 1.0,
                 op=m.OP_VARCOEF_NODAL if k is not None else m.OP_LAPLACE, k=dev(k) if k is not None else None)
    s = m.Solver(p)
    try:
        fused = m.mg_tile_config(s.ctx, 0, 6)[1] > 0
        u = dev(u0)
        st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
        return st, cyc, np.array(hist), host(u), fused
    finally:
        s.close()


CASES = [
    # dim, n, coefficient field, smoother, cycle, nu1, nu2
    (3, 65, False, RB, V, 2, 2), (3, 33, True, RB, V, 2, 2), (3, 33, False, JAC, V, 2, 2),
    (3, 17, False, SYM, W, 2, 2), (3, 33, True, JAC, F, 2, 2), (3, 129, False, RB, V, 2, 2),
    (3, 65, False, RB, V, 1, 1), (3, 33, False, RB, V, 3, 1), (2, 257, False, RB, V, 2, 2),
    (2, 129, True, JAC, F, 2, 2), (2, 65, False, SYM, W, 1, 2), (2, 1025, False, RB, V, 2, 2),
]


@pytest.mark.parametrize("dim,n,varcoef,smoother,cycle,nu1,nu2", CASES)
def test_fused_norm_solve_matches_oracle_and_separate_pass(dim, n, varcoef, smoother, cycle, nu1, nu2, dev_ok,
                                                           monkeypatch):
    f = inputs.uniform_rhs(dim, n, 71)
    k = inputs.varcoef_k(n, 72, dim=dim) if varcoef else None
    u0 = np.zeros_like(f)
    omega = 0.8 if smoother == JAC else 1.0
    ue, he, rce = oracle.solve(u0, f, tol=1e-10, max_cycles=30, smoother=smoother, omega=omega, nu1=nu1, nu2=nu2,
                               k=k, cycle=cycle)
    st1, c1, h1, u1, fused = gpu_solve(dim, n, f, u0, k, smoother, cycle, nu1, nu2)
    assert fused
    monkeypatch.setenv("MG_NO_FUSED_NORM", "1")
    st0, c0, h0, u0g, fused0 = gpu_solve(dim, n, f, u0, k, smoother, cycle, nu1, nu2)
    assert not fused0
    assert st1 == st0 == rce == 0
    assert c1 == c0 == len(he) - 1
    rt = norm_rtol(dim, n)
    np.testing.assert_allclose(h1, he, rtol=rt, atol=0)
    np.testing.assert_allclose(h1, h0, rtol=rt, atol=0)
    assert np.array_equal(u1, ue)
    assert np.array_equal(u0g, ue)


@pytest.mark.parametrize("dim,n,varcoef", [(3, 33, False), (3, 17, True), (2, 129, False)])
def test_fused_norm_of_a_nonzero_guess(dim, n, varcoef, dev_ok):
    """rho_0 comes from the first cycle's first sweep, on an arbitrary
    iterate; max_cycles 0 and 1 end the solve after that sweep and after the
    first cycle's norm, leaving u as the last cycle left it."""
    f = inputs.uniform_rhs(dim, n, 73)
    k = inputs.varcoef_k(n, 74, dim=dim) if varcoef else None
    u0 = inputs.zero_boundary(inputs.random_guess(dim, n, 75))
    rho0 = oracle.residual_norm(u0, f, k)
    st, cyc, h, u, fused = gpu_solve(dim, n, f, u0, k, max_cycles=0)
    assert fused and cyc == 0 and st == mg().MG_ENOTCONV
    assert h[0] == pytest.approx(rho0, rel=norm_rtol(dim, n))
    assert np.array_equal(u, u0)
    st, cyc, h, u, _ = gpu_solve(dim, n, f, u0, k, max_cycles=1, tol=0.0)
    ue, he, _ = oracle.solve(u0, f, tol=0.0, max_cycles=1, k=k)
    assert cyc == 1 and st == mg().MG_ENOTCONV
    np.testing.assert_allclose(h, he, rtol=norm_rtol(dim, n), atol=0)
    assert np.array_equal(u, ue)


def test_fused_norm_stops_on_the_cycle_that_converged(dev_ok):
    """A tolerance met after a few cycles: the extra first sweep that gave the
    last norm does not reach u."""
    dim, n = 3, 65
    f = inputs.uniform_rhs(dim, n, 76)
    u0 = np.zeros_like(f)
    ue, he, rc = oracle.solve(u0, f, tol=1e-4, max_cycles=30)
    st, cyc, h, u, fused = gpu_solve(dim, n, f, u0, tol=1e-4)
    assert fused and st == rc == 0 and cyc == len(he) - 1 < 10
    np.testing.assert_allclose(h, he, rtol=norm_rtol(dim, n), atol=0)
    assert np.array_equal(u, ue)


def test_fused_norm_full_size_513(dev_ok, monkeypatch):
    """513^3 in the tuned launch shapes: two cycles with the norm fused and
    with the separate pass give the same field bit for bit and the same norms
    to the summation-order bound."""
    import torch

    m = mg()
    dim, n = 3, 513
    f = dev(inputs.uniform_rhs(dim, n, 77))
    out = []
    for env in (None, "1"):
        if env:
            monkeypatch.setenv("MG_NO_FUSED_NORM", env)
        s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP64))
        try:
            fused = m.mg_tile_config(s.ctx, 0, 6)[1] > 0
            u = torch.zeros_like(f)
            st, cyc, hist = s.solve(u, f, tol=0.0, max_cycles=2)
            torch.cuda.synchronize()
            out.append((fused, cyc, np.array(hist), u))
        finally:
            s.close()
    assert out[0][0] and not out[1][0]
    assert out[0][1] == out[1][1] == 2
    np.testing.assert_allclose(out[0][2], out[1][2], rtol=norm_rtol(dim, n), atol=0)
    assert torch.equal(out[0][3], out[1][3])
    # the first norm is that of f (u0 = 0) on the inner nodes
    fi = f[1:-1, 1:-1, 1:-1]
    assert out[0][2][0] == pytest.approx(float(torch.linalg.vector_norm(fi)), rel=norm_rtol(dim, n))


def test_tile_config_family_6(dev_ok, monkeypatch):
    m = mg()
    s = m.Solver(m.Params(dim=3, n=65, precision=m.PREC_FP64))
    try:
        by, zc, pd, wv = m.mg_tile_config(s.ctx, 0, 6)
        assert by in (8, 16, 32) and zc > 0 and wv in (4, 8) and pd in (1, 2)
        with pytest.raises(m.MGError):
            m.mg_tile_config(s.ctx, 1, 6)
    finally:
        s.close()
    s = m.Solver(m.Params(dim=3, n=65, precision=m.PREC_FP32_IR))
    try:
        assert m.mg_tile_config(s.ctx, 0, 6) == (0, 0, 0, 0)
    finally:
        s.close()
    monkeypatch.setenv("MG_NO_FUSED_NORM", "1")
    s = m.Solver(m.Params(dim=2, n=65, precision=m.PREC_FP64))
    try:
        assert m.mg_tile_config(s.ctx, 0, 6) == (0, 0, 0, 0)
    finally:
        s.close()
