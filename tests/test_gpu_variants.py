"""Parity of the cycle and smoother variants with the CPU oracle: the
symmetric red-black smoother (post-smoothing sweeps relax black first), the
W- and F-cycles (two recursive calls per level; F: an F-cycle then a
V-cycle), and conjugate gradients on a coarsest level with more than one
unknown (Algorithm 1: "direct solver or CG").  Per-point arithmetic, CG inner
products (per x-row, then the rows in order) and the recursion order are the
same on both sides, so fields are compared bit for bit and solve histories to
1e-12 relative per cycle.
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


def same(a, b):
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    if a.dtype == np.float16:
        return np.array_equal(a.view(np.uint16), b.view(np.uint16))
    return np.array_equal(a, b)


def arrays(dim, n, dt, seed, varcoef=False):
    if dt == np.float16:
        c = float((n - 1) ** 2)
        u = (inputs.random_guess(dim, n, 700 + seed) * (8.0 / c)).astype(dt)
        f = (inputs.uniform_rhs(dim, n, 800 + seed) * 12.0).astype(dt)
    else:
        u = inputs.random_guess(dim, n, 700 + seed).astype(dt)
        f = (inputs.uniform_rhs(dim, n, 800 + seed) * 50.0).astype(dt)
    k = inputs.varcoef_k(n, 900 + seed, dim=dim).astype(dt) if varcoef else None
    return u, f, k


BLACK_FIRST = [
    # dim, n, by, zchunk, prefetch, waves
    (2, 33, 16, 0, 0, 0), (2, 129, 0, 0, 0, 0), (2, 257, 32, 0, 0, 0), (3, 9, 8, 1, 2, 0), (3, 33, 0, 0, 2, 0),
    (3, 65, 32, 7, 2, 8), (3, 129, 16, 33, 1, 8), (3, 65, 8, 9, 1, 1), (3, 129, 12, 13, 2, 1), (3, 17, 16, 3, 1, 4),
]


@pytest.mark.parametrize("dim,n,by,zc,pd,wv", BLACK_FIRST)
@pytest.mark.parametrize("dt", [np.float64, np.float32, np.float16])
@pytest.mark.parametrize("fused", [False, True])
def test_black_first_sweep_bitwise(dim, n, by, zc, pd, wv, dt, fused, dev_ok):
    """The post-smoothing sweep of the symmetric smoother (black first), plain
    and with the coarse-grid correction fused in."""
    u, f, _ = arrays(dim, n, dt, n)
    over = (by > 8) if wv == 1 else (by // (wv or 4) > 4)
    if dt == np.float64 and dim == 3 and over:
        # beyond the FP64 register limit of the 3D sweeps: rejected before any launch
        with pytest.raises(mg().MGError) as ei:
            mg().mg_level_smooth(dev(u), dev(f), dev(np.zeros_like(u)), smoother=SYM, by=by, zchunk=zc, prefetch=pd,
                                 waves=wv)
        assert ei.value.code == mg().MG_EINVAL
        return
    ec = None
    start = u
    if fused:
        nc = (n - 1) // 2 + 1
        scale = 8.0 / (n - 1) ** 2 if dt == np.float16 else 1.0
        ec = (inputs.random_guess(dim, nc, 33 + n) * scale).astype(dt)
        start = oracle.prolong_correct(u, ec)
    expect = oracle.smooth(start, f, smoother=oracle.SMOOTH_RBGS_SYM)
    out = dev(np.zeros_like(u))
    mg().mg_level_smooth(dev(u), dev(f), out, smoother=SYM, ec=dev(ec) if fused else None, by=by, zchunk=zc,
                         prefetch=pd, waves=wv)
    assert same(host(out), expect)


@pytest.mark.parametrize("dim,n,dt,varcoef", [(2, 5, np.float64, False), (2, 9, np.float64, True),
                                              (2, 33, np.float64, False), (2, 65, np.float32, False),
                                              (2, 17, np.float32, True), (3, 5, np.float64, False),
                                              (3, 9, np.float64, True), (3, 17, np.float32, False),
                                              (3, 9, np.float32, True), (3, 3, np.float64, False)])
@pytest.mark.parametrize("iters", [0, 3])
def test_coarsest_cg_bitwise(dim, n, dt, varcoef, iters, dev_ok):
    _, f, k = arrays(dim, n, dt, 5 * n, varcoef)
    f = np.ascontiguousarray(f)
    expect = oracle.coarsest_cg(np.zeros_like(f), f, k=k, iters=iters)
    u = dev(np.full(f.shape, 7.0, dtype=dt))  # overwritten, boundary included
    mg().mg_level_coarsest_cg(u, dev(f), k=dev(k) if varcoef else None, iters=iters)
    assert same(host(u), expect)


def test_coarsest_cg_size_limits(dev_ok):
    m = mg()
    f = np.zeros((17,) * 3)
    with pytest.raises(m.MGError) as ei:
        m.mg_level_coarsest_cg(dev(np.zeros_like(f)), dev(f))
    assert ei.value.code == m.MG_ENOTSUP


def solve(dim, n, f, precision, smoother=RB, cycle=V, coarse_n=0, cg_iters=0, k=None, tol=1e-9, max_cycles=40):
    m = mg()
    p = m.Params(dim=dim, n=n, smoother=smoother, precision=precision, cycle=cycle, coarse_n=coarse_n,
                 cg_iters=cg_iters, op=m.OP_VARCOEF_NODAL if k is not None else m.OP_LAPLACE,
                 k=dev(k) if k is not None else None)
    s = m.Solver(p)
    u = dev(np.zeros_like(f))
    st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
    out = host(u)
    s.close()
    return st, cyc, np.array(hist), out


SOLVES = [
    # dim, n, precision, smoother, cycle, coarse_n, varcoef
    (2, 129, 0, SYM, V, 0, False), (3, 65, 0, SYM, V, 0, False), (3, 33, 1, SYM, V, 0, True),
    (2, 65, 0, RB, W, 0, False), (3, 33, 0, JAC, W, 0, False), (2, 257, 1, SYM, W, 0, False),
    (3, 65, 1, RB, W, 0, False), (2, 129, 0, RB, F, 0, True), (3, 33, 1, SYM, F, 0, False),
    (2, 129, 0, RB, V, 17, False), (2, 257, 0, SYM, W, 33, False), (3, 33, 0, RB, V, 9, True),
    (3, 65, 1, RB, V, 17, False), (2, 129, 1, JAC, F, 65, False), (3, 65, 1, SYM, F, 9, False),
    (2, 17, 0, RB, V, 17, False), (2, 129, 2, SYM, W, 0, False), (3, 33, 2, RB, F, 9, False),
    (3, 65, 2, SYM, V, 17, False),
]


@pytest.mark.parametrize("dim,n,precision,smoother,cycle,coarse_n,varcoef", SOLVES)
def test_variant_solve_matches_oracle(dim, n, precision, smoother, cycle, coarse_n, varcoef, dev_ok):
    """Full solves with the variants, FP64, FP32-in-FP64 and binary16-in-FP64
    refinement; the 17-node grid with coarse_n 17 is one plain CG solve."""
    f = inputs.uniform_rhs(dim, n, 61)
    k = inputs.varcoef_k(n, 62, dim=dim) if varcoef else None
    omega = 0.8 if smoother == JAC else 1.0
    kw = dict(tol=1e-9, max_cycles=40, smoother=smoother, omega=omega, k=k, cycle=cycle,
              coarse_n=coarse_n if coarse_n else 3)
    ref = {0: oracle.solve, 1: oracle.solve_ir_f32, 2: oracle.solve_ir_f16}[precision]
    u_exp, h_exp, rc = ref(np.zeros_like(f), f, **kw)
    st, cyc, h, u = solve(dim, n, f, precision, smoother=smoother, cycle=cycle, coarse_n=coarse_n, k=k)
    assert cyc == len(h_exp) - 1 and st == rc
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert same(u, u_exp)


def test_symmetric_v_cycle_tail_equals_level_by_level(dev_ok, monkeypatch):
    """The coarse tail kernel relaxes black first after the correction too."""
    f = inputs.uniform_rhs(3, 65, 71)
    monkeypatch.setenv("MG_NO_TAIL", "1")
    st0, c0, h0, u0 = solve(3, 65, f, 1, smoother=SYM)
    monkeypatch.delenv("MG_NO_TAIL")
    st1, c1, h1, u1 = solve(3, 65, f, 1, smoother=SYM)
    assert c0 == c1 and same(u0, u1)


def test_variant_parameters_rejected(dev_ok):
    m = mg()
    for kw, code in [(dict(cycle=3), m.MG_EINVAL), (dict(coarse_n=7), m.MG_EINVAL), (dict(coarse_n=65), m.MG_EINVAL),
                     (dict(coarse_n=17), m.MG_ENOTSUP), (dict(cg_iters=-1), m.MG_EINVAL), (dict(smoother=3), m.MG_EINVAL)]:
        with pytest.raises(m.MGError) as ei:
            m.Solver(m.Params(dim=3, n=33, **kw))  # FP64: CG coarsest edge at most 9 in 3D
        assert ei.value.code == code, kw
    with pytest.raises(m.MGError) as ei:
        m.mg_batch_setup([m.Params(dim=2, n=65, precision=m.PREC_FP32_IR, cycle=W)])
    assert ei.value.code == m.MG_ENOTSUP
