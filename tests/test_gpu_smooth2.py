"""Parity of the first two pre-smoothing sweeps from a zero iterate fused in
one launch (Algorithm 1: presmoothing from the zero coarse-grid guess) with
the CPU oracle's two sweeps, bit for bit, in FP32 and in binary16 storage
(FP32 arithmetic), over grid sizes that give one or many tiles, ragged last
tiles in x, y and z, both tile heights and several chunk depths; and whole
solves with the fused launch forced on and off.
"""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


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
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    if a.dtype == np.float16:
        return np.array_equal(a.view(np.uint16), b.view(np.uint16))
    return np.array_equal(a, b)


def rhs(n, dt, seed):
    if dt == np.float16:
        return (inputs.uniform_rhs(3, n, 960 + seed) * 12.0).astype(dt)
    return (inputs.uniform_rhs(3, n, 960 + seed) * 50.0).astype(dt)


@pytest.mark.parametrize("n", [5, 9, 17, 33, 65, 129])
@pytest.mark.parametrize("by", [12, 16])
@pytest.mark.parametrize("zc", [1, 2, 3, 7, 16])
@pytest.mark.parametrize("dt", [np.float32, np.float16])
def test_two_sweeps_from_zero_bitwise(n, by, zc, dt, dev_ok):
    f = rhs(n, dt, n + by + zc)
    u1 = oracle.smooth(np.zeros_like(f), f, oracle.SMOOTH_RBGS, 1.0)
    expect = oracle.smooth(u1, f, oracle.SMOOTH_RBGS, 1.0)
    for order in (0, 1):
        out = dev(np.zeros_like(f))
        mg().mg_level_smooth2_zero(dev(f), out, by=by, zchunk=zc, order=order)
        assert same(host(out), expect), (order,)


def test_two_sweeps_equal_the_two_kernels_at_513(dev_ok):
    """513^3 FP32: the fused launch equals the zero-iterate sweep followed by
    the plain sweep of the tuned path's kernels (both pinned above against
    the oracle)."""
    import torch

    m = mg()
    n = 513
    f = dev(rhs(n, np.float32, 1))
    t = torch.zeros_like(f)
    u = torch.zeros_like(f)
    m.mg_level_smooth(t, f, t, zero_guess=True)
    m.mg_level_smooth(t, f, u)
    for by, zc in ((12, 16), (16, 32)):
        out = torch.zeros_like(f)
        m.mg_level_smooth2_zero(f, out, by=by, zchunk=zc)
        torch.cuda.synchronize()
        assert torch.equal(out, u), (by, zc)


@pytest.mark.parametrize("n,precision", [(65, 1), (129, 1), (65, 2), (257, 1)])
def test_solve_with_and_without_the_fused_sweeps(n, precision, dev_ok, monkeypatch):
    """FP32-IR / binary16-IR solves as autotuned, with the fused launch forced
    on every level it applies to, and switched off: every history and field
    equals the oracle's."""
    m = mg()
    f = inputs.uniform_rhs(3, n, 5)
    solve = oracle.solve_ir_f32 if precision == 1 else oracle.solve_ir_f16
    res = solve(np.zeros_like(f), f, tol=1e-8, max_cycles=30)
    ue, he = res[0], res[1]
    for env in ({}, {"MG_FUSED_SMOOTH2": "1"}, {"MG_NO_FUSED_SMOOTH2": "1"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        s = m.Solver(m.Params(dim=3, n=n, precision=precision))
        try:
            u = dev(np.zeros_like(f))
            st, cyc, hist = s.solve(u, dev(f), tol=1e-8, max_cycles=30)
            assert cyc == len(he) - 1
            np.testing.assert_allclose(hist, he, rtol=1e-12, atol=0)
            assert np.array_equal(host(u), ue)
        finally:
            s.close()
        for k in env:
            monkeypatch.delenv(k)


def test_two_sweeps_reject_bad_arguments(dev_ok):
    import torch

    m = mg()
    f = torch.zeros((9, 9, 9), dtype=torch.float32, device="cuda")
    for kw in (dict(by=8), dict(by=32), dict(zchunk=0), dict(order=2)):
        with pytest.raises(m.MGError):
            m.mg_level_smooth2_zero(f, f.clone(), **kw)
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_zero(f, f)  # in place
    f64 = torch.zeros((9, 9, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_zero(f64, f64.clone())  # FP64 is not built
    f2 = torch.zeros((9, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_zero(f2, f2.clone())  # 3D only
