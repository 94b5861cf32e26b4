"""Parity of the last pre-smoothing sweep fused with the residual and full
weighting (Algorithm 1: presmoothing, residual, restriction) with the CPU
oracle: one red-first red-black sweep and the restriction of the residual of
its result, bit for bit, in FP32 and in binary16 storage (FP32 arithmetic),
over grid sizes that give one or many tiles, ragged last tiles in x, y and z,
and every chunk depth; and whole solves with the fused kernel forced on and
off.
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


def arrays(n, dt, seed):
    if dt == np.float16:
        c = float((n - 1) ** 2)
        u = (inputs.random_guess(3, n, 900 + seed) * (8.0 / c)).astype(dt)
        f = (inputs.uniform_rhs(3, n, 950 + seed) * 12.0).astype(dt)
    else:
        u = inputs.random_guess(3, n, 900 + seed).astype(dt)
        f = (inputs.uniform_rhs(3, n, 950 + seed) * 50.0).astype(dt)
    return u, f


@pytest.mark.parametrize("n", [5, 9, 17, 33, 65, 129])
@pytest.mark.parametrize("zc", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("dt", [np.float32, np.float16])
def test_fused_sweep_restrict_bitwise(n, zc, order, dt, dev_ok):
    u, f = arrays(n, dt, n + zc)
    expect_u = oracle.smooth(u, f, oracle.SMOOTH_RBGS, 1.0)
    r = oracle.residual(expect_u, f)
    expect_fc = oracle.restrict(r, out_dtype=np.float16) if dt == np.float16 else oracle.restrict(r)
    nc = (n - 1) // 2 + 1
    uo = dev(np.zeros_like(u))
    fc = dev(np.zeros((nc,) * 3, dtype=dt))
    mg().mg_level_smooth_restrict(dev(u), dev(f), uo, fc, zchunk=zc, order=order)
    assert same(host(uo), expect_u)
    assert same(host(fc), expect_fc)


def test_fused_sweep_restrict_full_size_sampled(dev_ok):
    """513^3 FP32 in the solver's launch shape: the sweep result and the
    restricted residual at sampled coarse nodes against the oracle's formulas
    evaluated one node at a time on the GPU's own sweep output (which the
    smaller cases pin bit for bit)."""
    n = 513
    u, f = arrays(n, np.float32, 7)
    nc = (n - 1) // 2 + 1
    uo = dev(np.zeros_like(u))
    fc = dev(np.zeros((nc,) * 3, dtype=np.float32))
    mg().mg_level_smooth_restrict(dev(u), dev(f), uo, fc, zchunk=8, order=0)
    us, fcs = host(uo), host(fc)
    ref = dev(np.zeros_like(u))
    mg().mg_level_smooth(dev(u), dev(f), ref)  # the separate sweep kernel (pinned against the oracle)
    assert np.array_equal(us, host(ref))
    rng = np.random.default_rng(3)
    for _ in range(40):
        K, J, I = (int(x) for x in rng.integers(1, nc - 1, 3))
        sub = us[2 * K - 2:2 * K + 3, 2 * J - 2:2 * J + 3, 2 * I - 2:2 * I + 3].copy()
        fsub = f[2 * K - 2:2 * K + 3, 2 * J - 2:2 * J + 3, 2 * I - 2:2 * I + 3].copy()
        # residual of the 3x3x3 fine nodes around 2I with the level's h
        c = np.float32((n - 1) ** 2)
        r = np.zeros((3, 3, 3), np.float32)
        for a in range(3):
            for b in range(3):
                for e in range(3):
                    z, y, x = a + 1, b + 1, e + 1
                    s = ((sub[z, y, x - 1] + sub[z, y, x + 1]) + (sub[z, y - 1, x] + sub[z, y + 1, x])) + \
                        (sub[z - 1, y, x] + sub[z + 1, y, x])
                    r[a, b, e] = fsub[z, y, x] - c * (np.float32(6) * sub[z, y, x] - s)
        faces = ((r[1, 1, 0] + r[1, 1, 2]) + (r[1, 0, 1] + r[1, 2, 1])) + (r[0, 1, 1] + r[2, 1, 1])
        exy = (r[1, 0, 0] + r[1, 0, 2]) + (r[1, 2, 0] + r[1, 2, 2])
        exz = (r[0, 1, 0] + r[0, 1, 2]) + (r[2, 1, 0] + r[2, 1, 2])
        eyz = (r[0, 0, 1] + r[0, 2, 1]) + (r[2, 0, 1] + r[2, 2, 1])
        edges = (exy + exz) + eyz
        cz0 = (r[0, 0, 0] + r[0, 0, 2]) + (r[0, 2, 0] + r[0, 2, 2])
        cz1 = (r[2, 0, 0] + r[2, 0, 2]) + (r[2, 2, 0] + r[2, 2, 2])
        v = ((np.float32(0.125) * r[1, 1, 1] + np.float32(0.0625) * faces) + np.float32(0.03125) * edges) + \
            np.float32(0.015625) * (cz0 + cz1)
        assert fcs[K, J, I] == v, (K, J, I)


@pytest.mark.parametrize("n,precision", [(65, 1), (129, 1), (65, 2), (257, 1)])
def test_solve_with_and_without_fusion_equal_oracle(n, precision, dev_ok, monkeypatch):
    """Whole FP32-IR / binary16-IR solves as autotuned, with the fused kernel
    forced on every tuned level, and with it switched off: every history and
    field equals the oracle's."""
    m = mg()
    f = inputs.uniform_rhs(3, n, 5)
    solve = oracle.solve_ir_f32 if precision == 1 else oracle.solve_ir_f16
    res = solve(np.zeros_like(f), f, tol=1e-8, max_cycles=30)
    ue, he = res[0], res[1]
    for env in ({}, {"MG_FUSED_RESTRICT": "1"}, {"MG_NO_FUSED_RESTRICT": "1"}):
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


def test_fused_rejects_bad_arguments(dev_ok):
    import torch

    m = mg()
    u = torch.zeros((9, 9, 9), dtype=torch.float32, device="cuda")
    fc = torch.zeros((5, 5, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(m.MGError):
        m.mg_level_smooth_restrict(u, u, u, fc)  # in place
    with pytest.raises(m.MGError):
        m.mg_level_smooth_restrict(u, u.clone(), u.clone(), fc, zchunk=0)
    u64 = torch.zeros((9, 9, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(m.MGError):
        m.mg_level_smooth_restrict(u64, u64.clone(), u64.clone(), fc.double())  # FP64 is not built
