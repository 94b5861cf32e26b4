"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (autotuned tile geometry, graph-captured solve chunks), plus
the degenerate and the largest accepted grids.

* 513^3 Poisson, FP32 V(2,2) cycles in FP64 refinement to 1e-8: the whole
  solve is compared with the oracle's (history to 1e-12 per step, field bit for
  bit).
* 257^3 variable-coefficient problem (k in [1, 100]), same solver: same bar.
* 512 batched 2D grids with edges 65..1025: every instance is compared with
  the oracle (refinement steps, field bit for bit).
* n = 3 (one unknown: the coarsest solve alone) and a zero right-hand side.
* The largest grids the library accepts (2D 32769^2 and 3D 1025^3, each about
  1.07e9 nodes): the oracle's FP64 residual of the GPU answer is checked against
  the tolerance and against the norm the GPU reported.
"""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def gpu_solve(dim, n, f, precision, tol, max_cycles=50, k=None):
    m = mg()
    kd = dev(k) if k is not None else None
    p = m.Params(dim=dim, n=n, precision=precision, k=kd, op=m.OP_VARCOEF_NODAL if k is not None else m.OP_LAPLACE)
    s = m.Solver(p)
    u = dev(np.zeros_like(f))
    st, cyc, hist = s.solve(u, dev(f), tol=tol, max_cycles=max_cycles)
    out = host(u)
    s.close()
    return st, cyc, np.array(hist), out


def test_poisson3d_513_fp32ir_matches_oracle(dev_ok):
    f = inputs.uniform_rhs(3, 513, 0)
    print("[fullsize] 513^3 FP32-IR: GPU solve", flush=True)
    st, cyc, h, u = gpu_solve(3, 513, f, 1, 1e-8)
    assert st == 0
    print(f"[fullsize] 513^3 FP32-IR: {cyc} steps; oracle solve", flush=True)
    u_exp, h_exp, rc = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=50)
    assert rc == 0 and cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert np.array_equal(u, u_exp)


def test_varcoef3d_257_fp32ir_matches_oracle(dev_ok):
    k = inputs.varcoef_k(257, 1, dim=3)
    f = inputs.uniform_rhs(3, 257, 2)
    assert k.min() == pytest.approx(1.0) and k.max() == pytest.approx(100.0)
    st, cyc, h, u = gpu_solve(3, 257, f, 1, 1e-8, k=k)
    assert st == 0
    u_exp, h_exp, rc = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=50, k=k)
    assert rc == 0 and cyc == len(h_exp) - 1
    np.testing.assert_allclose(h, h_exp, rtol=1e-12, atol=0)
    assert np.array_equal(u, u_exp)


def test_batched_512_grids_against_oracle(dev_ok):
    """Every one of the 512 instances: refinement steps and field bit for bit."""
    import torch

    m = mg()
    edges, fs = inputs.batch_problem()
    assert len(edges) == 512
    ctx = m.mg_batch_setup([m.Params(dim=2, n=int(n), precision=m.PREC_FP32_IR) for n in edges])
    us = [torch.zeros((int(n), int(n)), dtype=torch.float64, device="cuda") for n in edges]
    fd = [dev(f) for f in fs]
    print("[fullsize] 512-grid batch: GPU solve", flush=True)
    st, cyc, stt = m.mg_batch_solve(ctx, us, fd, tol=1e-8, max_cycles=50)
    torch.cuda.synchronize()
    m.mg_destroy(ctx)
    assert st == 0 and all(x == 0 for x in stt)
    print("[fullsize] 512-grid batch: oracle solves", flush=True)
    bad = []
    for i in range(512):
        u_ref, h_ref, rc = oracle.solve_ir_f32(np.zeros_like(fs[i]), fs[i], tol=1e-8, max_cycles=50)
        if rc != 0 or cyc[i] != len(h_ref) - 1 or not np.array_equal(us[i].cpu().numpy(), u_ref):
            bad.append((i, int(edges[i])))
    assert not bad, f"instances differing from the oracle: {bad[:10]} ({len(bad)} in all)"


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_single_unknown_grid(dim, precision, dev_ok):
    """n = 3: the hierarchy is the coarsest level alone and one cycle is exact."""
    f = np.zeros((3,) * dim)
    f[(1,) * dim] = 3.0
    st, cyc, h, u = gpu_solve(dim, 3, f, precision, 1e-12)
    expect = np.zeros_like(f)
    expect[(1,) * dim] = 3.0 / (2 * dim * 4.0)  # f / diag, diag = 2d / h^2 with h = 1/2
    assert st == 0 and cyc == 1 and h[-1] == 0.0
    assert np.array_equal(u, expect)


@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33)])
@pytest.mark.parametrize("precision", [0, 1])
def test_zero_rhs_is_converged_at_once(dim, n, precision, dev_ok):
    f = np.zeros((n,) * dim)
    st, cyc, h, u = gpu_solve(dim, n, f, precision, 1e-8)
    assert st == 0 and cyc == 0 and h[0] == 0.0
    assert not u.any()


def test_sizes_beyond_the_limits_are_rejected(dev_ok):
    m = mg()
    for dim, n in ((2, 65537), (3, 2049)):
        with pytest.raises(m.MGError) as ei:
            m.Solver(m.Params(dim=dim, n=n))
        assert ei.value.code == m.MG_EINVAL


@pytest.mark.parametrize("dim,n", [(3, 1025), (2, 32769)])
def test_largest_grids_converge(dim, n, dev_ok):
    """About 1.07e9 nodes: the oracle's FP64 residual of the GPU answer meets the
    tolerance and matches the last norm of the GPU's history."""
    import torch

    m = mg()
    f = inputs.uniform_rhs(dim, n, 9)
    print(f"[fullsize] largest grid dim={dim} n={n}: GPU solve", flush=True)
    s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR))
    fd = dev(f)
    u = torch.zeros_like(fd)
    st, cyc, hist = s.solve(u, fd, tol=1e-8, max_cycles=50)
    s.close()
    del fd
    assert st == 0
    uh = host(u)
    del u
    torch.cuda.empty_cache()
    print(f"[fullsize] largest grid: {cyc} steps; oracle residual", flush=True)
    r0 = oracle.residual_norm(np.zeros_like(f), f)
    r = oracle.residual_norm(uh, f)
    # The two sides sum ~1e9 squares in different orders: the oracle row by row
    # (or plane by plane) then over rows, the GPU per tile then over tiles.  With
    # at most ~6.6e4 sequential additions on either side the relative difference
    # of the sums is bounded by ~6.6e4 * 2^-53 = 7e-12, halved by the square root.
    assert r0 == pytest.approx(hist[0], rel=1e-10)
    assert r == pytest.approx(hist[-1], rel=1e-9)
    assert r <= 1e-8 * r0
