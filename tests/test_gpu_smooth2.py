"""Parity of the first two pre-smoothing sweeps from a zero iterate fused in
one launch (Algorithm 1: presmoothing from the zero coarse-grid guess) with
the CPU oracle's two sweeps, bit for bit, in FP32 and in binary16 storage
(FP32 arithmetic), 2D and 3D, over grid sizes that give one or many tiles,
ragged last tiles in x, y and z, both 3D tile heights and several chunk
depths; and whole solves and batches with the fused launch forced on and off.
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


@pytest.mark.parametrize("n", [5, 9, 33, 65, 129, 257, 513])
@pytest.mark.parametrize("yc", [1, 3, 16, 64])
@pytest.mark.parametrize("dt", [np.float32, np.float16])
def test_two_sweeps_from_zero_bitwise_2d(n, yc, dt, dev_ok):
    """2D: 64-wide strips (58 written nodes) marching chunks of yc rows, four
    chunks per workgroup (ragged strips, chunks and workgroups)."""
    if dt == np.float16:
        f = (inputs.uniform_rhs(2, n, 970 + n + yc) * 12.0).astype(dt)
    else:
        f = (inputs.uniform_rhs(2, n, 970 + n + yc) * 50.0).astype(dt)
    u1 = oracle.smooth(np.zeros_like(f), f, oracle.SMOOTH_RBGS, 1.0)
    expect = oracle.smooth(u1, f, oracle.SMOOTH_RBGS, 1.0)
    for order in (0, 1):
        out = dev(np.zeros_like(f))
        mg().mg_level_smooth2_zero(dev(f), out, zchunk=yc, order=order)
        assert same(host(out), expect), (order,)


@pytest.mark.parametrize("n", [5, 9, 33, 65, 129, 257, 513])
@pytest.mark.parametrize("yc", [1, 3, 16, 64])
@pytest.mark.parametrize("dt", [np.float32, np.float16])
@pytest.mark.parametrize("smoother", [0, 2])
def test_two_post_sweeps_with_correction_bitwise_2d(n, yc, dt, smoother, dev_ok):
    """2D: the bilinear correction and two red-black sweeps (red first, or
    black first as the symmetric smoother's post-smoothing) in one launch,
    against the oracle's correction and two sweeps."""
    nc = (n - 1) // 2 + 1
    if dt == np.float16:
        scale = 8.0 / (n - 1) ** 2
        u = (inputs.random_guess(2, n, 980 + n) * scale).astype(dt)
        f = (inputs.uniform_rhs(2, n, 981 + yc) * 12.0).astype(dt)
        ec = (inputs.random_guess(2, nc, 982 + n) * scale).astype(dt)
    else:
        u = inputs.random_guess(2, n, 980 + n).astype(dt)
        f = (inputs.uniform_rhs(2, n, 981 + yc) * 50.0).astype(dt)
        ec = inputs.random_guess(2, nc, 982 + n).astype(dt)
    sm = oracle.SMOOTH_RBGS_SYM if smoother == 2 else oracle.SMOOTH_RBGS
    u1 = oracle.smooth(oracle.prolong_correct(u, ec), f, smoother=sm)
    expect = oracle.smooth(u1, f, smoother=sm)
    for order in (0, 1):
        out = dev(np.zeros_like(u))
        mg().mg_level_smooth2_correct(dev(u), dev(f), dev(ec), out, smoother=smoother, zchunk=yc, order=order)
        got = host(out)
        # the boundary is not written (zero in out, as loaded in the oracle's copy)
        inner = (slice(1, -1),) * 2
        assert same(np.ascontiguousarray(got[inner]), np.ascontiguousarray(expect[inner])), (order,)


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


@pytest.mark.parametrize("dim,n,precision", [(3, 65, 1), (3, 129, 1), (3, 65, 2), (3, 257, 1), (2, 513, 1),
                                             (2, 1025, 1), (2, 257, 2)])
def test_solve_with_and_without_the_fused_sweeps(dim, n, precision, dev_ok, monkeypatch):
    """FP32-IR / binary16-IR solves as autotuned, with the fused launch forced
    on every level it applies to, and switched off: every history and field
    equals the oracle's."""
    m = mg()
    f = inputs.uniform_rhs(dim, n, 5)
    solve = oracle.solve_ir_f32 if precision == 1 else oracle.solve_ir_f16
    res = solve(np.zeros_like(f), f, tol=1e-8, max_cycles=30)
    ue, he = res[0], res[1]
    for env in ({}, {"MG_FUSED_SMOOTH2": "1", "MG_FUSED_POST2": "1"}, {"MG_NO_FUSED_SMOOTH2": "1"},
                {"MG_NO_FUSED_POST2": "1"}, {"MG_FUSED_POST2": "1", "MG_NO_FUSED_SMOOTH2": "1"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        s = m.Solver(m.Params(dim=dim, n=n, precision=precision))
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


def test_symmetric_smoother_solves_with_the_fused_sweeps(dev_ok, monkeypatch):
    """The symmetric red-black smoother (black first after the correction)
    with both fused pairs forced on, V and W cycles, equals the oracle."""
    m = mg()
    f = inputs.uniform_rhs(2, 257, 8)
    monkeypatch.setenv("MG_FUSED_SMOOTH2", "1")
    monkeypatch.setenv("MG_FUSED_POST2", "1")
    for cycle in (m.CYCLE_V, m.CYCLE_W):
        ue, he, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=30, smoother=oracle.SMOOTH_RBGS_SYM,
                                        cycle=cycle)
        s = m.Solver(m.Params(dim=2, n=257, precision=m.PREC_FP32_IR, smoother=m.SMOOTH_RBGS_SYM, cycle=cycle))
        try:
            u = dev(np.zeros_like(f))
            st, cyc, hist = s.solve(u, dev(f), tol=1e-8, max_cycles=30)
            assert cyc == len(he) - 1
            np.testing.assert_allclose(hist, he, rtol=1e-12, atol=0)
            assert np.array_equal(host(u), ue)
        finally:
            s.close()


@pytest.mark.parametrize("dim,edges", [(2, [65, 129, 33, 257, 65, 9, 129, 513]), (3, [17, 33, 9, 65, 33])])
def test_batch_with_the_fused_sweeps_matches_oracle(dim, edges, dev_ok, monkeypatch):
    """Batched solves with the fused launch forced on every level equal the
    oracle's solves of each grid."""
    import torch

    m = mg()
    monkeypatch.setenv("MG_FUSED_SMOOTH2", "1")
    monkeypatch.setenv("MG_FUSED_POST2", "1")
    fs = [inputs.uniform_rhs(dim, n, 710 + i) for i, n in enumerate(edges)]
    ctx = m.mg_batch_setup([m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR) for n in edges])
    try:
        us = [dev(np.zeros_like(f)) for f in fs]
        st, cyc, stt = m.mg_batch_solve(ctx, us, [dev(f) for f in fs], tol=1e-8, max_cycles=40)
        assert st == 0 and all(x == 0 for x in stt)
        torch.cuda.synchronize()
        for i, f in enumerate(fs):
            u_ref, h_ref, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
            assert cyc[i] == len(h_ref) - 1
            assert np.array_equal(us[i].cpu().numpy(), u_ref)
    finally:
        m.mg_destroy(ctx)


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
        m.mg_level_smooth2_zero(f2, f2.clone(), zchunk=0)
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_zero(f2, f2)  # in place
    e2 = torch.zeros((5, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_correct(f2, f2.clone(), e2, f2)  # in place
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_correct(f2, f2.clone(), e2, f2.clone(), smoother=1)  # Jacobi is not built
    with pytest.raises(m.MGError):
        m.mg_level_smooth2_correct(f, f.clone(), torch.zeros((5, 5, 5), device="cuda"), f.clone())  # 2D only
