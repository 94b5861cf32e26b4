"""Batched and served solves: every instance's answer is bit-identical to
solving it alone (mg_solve, and the CPU oracle's FP32-in-FP64 refinement)."""

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


def alone(dim, n, f):
    m = mg()
    s = m.Solver(m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR))
    u = dev(np.zeros_like(f))
    st, cyc, hist = s.solve(u, dev(f), tol=1e-8, max_cycles=40)
    import torch

    torch.cuda.synchronize()
    out = u.cpu().numpy()
    s.close()
    return st, cyc, out


@pytest.mark.parametrize("dim,edges", [(2, [65, 129, 33, 257, 65, 9, 129, 513]), (3, [17, 33, 9, 65, 33])])
def test_batch_matches_alone_and_oracle(dim, edges, dev_ok):
    import torch

    m = mg()
    fs = [inputs.uniform_rhs(dim, n, 700 + i) for i, n in enumerate(edges)]
    ctx = m.mg_batch_setup([m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR) for n in edges])
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, stt = m.mg_batch_solve(ctx, us, [dev(f) for f in fs], tol=1e-8, max_cycles=40)
    assert st == 0 and all(x == 0 for x in stt)
    torch.cuda.synchronize()
    for i, (n, f) in enumerate(zip(edges, fs)):
        got = us[i].cpu().numpy()
        u_ref, h_ref, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
        assert cyc[i] == len(h_ref) - 1
        assert np.array_equal(got, u_ref)
        st1, c1, u1 = alone(dim, n, f)
        assert c1 == cyc[i] and np.array_equal(u1, got)
    # a second solve on the same context (same buffers, reset) repeats the answer
    for u in us:
        u.zero_()
    st2, cyc2, _ = m.mg_batch_solve(ctx, us, [dev(f) for f in fs], tol=1e-8, max_cycles=40)
    assert cyc2 == cyc
    m.mg_destroy(ctx)


@pytest.mark.parametrize("dim,edges", [(2, [65, 33, 129, 9, 257]), (3, [17, 33, 9, 65])])
def test_batch_jacobi_matches_oracle(dim, edges, dev_ok):
    """Batched weighted-Jacobi (omega 0.8) solves equal the oracle's refinement with the same smoother."""
    import torch

    m = mg()
    fs = [inputs.uniform_rhs(dim, n, 760 + i) for i, n in enumerate(edges)]
    ctx = m.mg_batch_setup([m.Params(dim=dim, n=n, precision=m.PREC_FP32_IR, smoother=m.SMOOTH_JACOBI)
                            for n in edges])
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, stt = m.mg_batch_solve(ctx, us, [dev(f) for f in fs], tol=1e-8, max_cycles=60)
    torch.cuda.synchronize()
    m.mg_destroy(ctx)
    assert st == 0 and all(x == 0 for x in stt)
    for i, f in enumerate(fs):
        u_ref, h_ref, rc = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=60,
                                               smoother=oracle.SMOOTH_JACOBI, omega=0.8)
        assert rc == 0 and cyc[i] == len(h_ref) - 1, i
        assert np.array_equal(us[i].cpu().numpy(), u_ref), i


def test_batch_rejects_mixed_solver_settings(dev_ok):
    m = mg()
    with pytest.raises(m.MGError):
        m.mg_batch_setup([m.Params(dim=2, n=65, precision=1), m.Params(dim=2, n=65, precision=1, nu1=1)])
    with pytest.raises(m.MGError) as ei:
        m.mg_batch_setup([m.Params(dim=2, n=65, precision=0)])
    assert ei.value.code == m.MG_ENOTSUP


def test_server_results_equal_alone_in_the_mix(dev_ok):
    """Requests that arrive while others run are admitted as slots and budget free up;
    each result equals the solve of that request alone."""
    m = mg()
    sp = m.ServerParams(hbm_budget_bytes=256 << 20, max_slots=3, max_n2d=257, max_n3d=33, tol=1e-8, max_cycles=40)
    ctx = m.mg_server_create(sp)
    reqs = [(2, 129, 1), (3, 33, 2), (2, 257, 3), (2, 65, 4), (3, 17, 5), (2, 129, 6), (2, 33, 7), (3, 33, 8),
            (2, 257, 9), (2, 65, 10)]
    f_of = {}
    pending = list(reqs)
    done = {}
    steps = 0
    # submit two at a time between steps: arrivals overlap running requests
    while pending or len(done) < len(reqs):
        for _ in range(2):
            if pending:
                dim, n, seed = pending.pop(0)
                f = inputs.uniform_rhs(dim, n, 900 + seed)
                rid = m.mg_server_submit(ctx, f)
                f_of[rid] = (dim, n, f)
        active, queued = m.mg_server_step(ctx)
        assert active <= 2 * sp.max_slots
        used, _, _ = m.mg_server_info(ctx)
        assert used <= sp.hbm_budget_bytes
        for rid in m.mg_server_poll(ctx):
            dim, n, f = f_of[rid]
            st, u, cyc, rr, lat = m.mg_server_fetch(ctx, rid, shape=f.shape)
            done[rid] = (st, u, cyc, rr)
        steps += 1
        assert steps < 500
    for rid, (st, u, cyc, rr) in done.items():
        dim, n, f = f_of[rid]
        assert st == 0 and rr <= 1e-8
        u_ref, h_ref, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
        assert cyc == len(h_ref) - 1
        assert np.array_equal(u, u_ref)
    m.mg_destroy(ctx)


def test_server_budget_blocks_then_admits(dev_ok):
    """A budget that fits one large request at a time serialises them without starving any."""
    m = mg()
    f = inputs.uniform_rhs(2, 513, 1)
    need = 513 * 513 * (24 + 4 * 3 * 4 // 3) + (1 << 20)
    sp = m.ServerParams(hbm_budget_bytes=need, max_slots=8, max_n2d=513, max_n3d=17, tol=1e-8, max_cycles=40)
    ctx = m.mg_server_create(sp)
    ids = [m.mg_server_submit(ctx, f) for _ in range(3)]
    finished = []
    for _ in range(200):
        active, queued = m.mg_server_step(ctx)
        assert active <= 1
        finished += m.mg_server_poll(ctx)
        if len(finished) == 3:
            break
    assert finished == ids  # arrival order, none overtaken
    for rid in ids:
        st, u, cyc, rr, lat = m.mg_server_fetch(ctx, rid)
        assert st == 0
    m.mg_destroy(ctx)


def test_server_many_requests_reusing_few_slots(dev_ok):
    """Forty requests through two slots per dimension, submitted in bursts of zero to
    three between steps, including zero right-hand sides (finished before the first
    cycle): slots and hierarchies are reused while earlier steps are still in flight,
    and every result equals the oracle's solve of that request alone."""
    m = mg()
    sp = m.ServerParams(hbm_budget_bytes=512 << 20, max_slots=2, max_n2d=129, max_n3d=17, tol=1e-8, max_cycles=40)
    ctx = m.mg_server_create(sp)
    rng = np.random.default_rng(21)
    sizes = [(2, 33), (2, 65), (2, 129), (3, 9), (3, 17)]
    reqs = []
    for i in range(40):
        dim, n = sizes[int(rng.integers(len(sizes)))]
        f = np.zeros((n,) * dim) if i % 13 == 5 else inputs.uniform_rhs(dim, n, 1200 + i)
        reqs.append(f)
    f_of, done, i, steps = {}, {}, 0, 0
    while i < len(reqs) or len(done) < len(reqs):
        for _ in range(int(rng.integers(0, 4))):
            if i < len(reqs):
                f_of[m.mg_server_submit(ctx, reqs[i])] = reqs[i]
                i += 1
        m.mg_server_step(ctx)
        for rid in m.mg_server_poll(ctx):
            st, u, cyc, rr, lat = m.mg_server_fetch(ctx, rid, shape=f_of[rid].shape)
            done[rid] = (st, u, cyc)
        steps += 1
        assert steps < 3000
    assert sorted(done) == sorted(f_of)
    for rid, (st, u, cyc) in done.items():
        f = f_of[rid]
        assert st == 0
        u_ref, h_ref, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
        assert cyc == len(h_ref) - 1, rid
        assert np.array_equal(u, u_ref), rid
    m.mg_destroy(ctx)


def test_server_mix_at_full_request_sizes(dev_ok):
    """The served mix at its full edge range (2D up to 2049^2, 3D up to 257^3):
    requests of every size arrive while others run, and each result equals the
    oracle's FP32-in-FP64 solve of that request alone, bit for bit."""
    m = mg()
    sp = m.ServerParams(hbm_budget_bytes=16 << 30, max_slots=4, max_n2d=2049, max_n3d=257, tol=1e-8, max_cycles=40)
    ctx = m.mg_server_create(sp)
    reqs = [(2, 2049, 1), (3, 257, 2), (2, 257, 3), (3, 33, 4), (2, 1025, 5), (3, 65, 6), (2, 513, 7),
            (3, 129, 8), (2, 2049, 9), (3, 257, 10)]
    pending = list(reqs)
    f_of, done, steps = {}, {}, 0
    while pending or len(done) < len(reqs):
        for _ in range(3):
            if pending:
                dim, n, seed = pending.pop(0)
                f = inputs.uniform_rhs(dim, n, 1500 + seed)
                f_of[m.mg_server_submit(ctx, f)] = f
        m.mg_server_step(ctx)
        for rid in m.mg_server_poll(ctx):
            st, u, cyc, rr, lat = m.mg_server_fetch(ctx, rid, shape=f_of[rid].shape)
            done[rid] = (st, u, cyc, rr)
        steps += 1
        assert steps < 2000
    m.mg_destroy(ctx)
    print(f"[serve] {len(done)} full-size requests served in {steps} steps; oracle solves", flush=True)
    for rid, (st, u, cyc, rr) in done.items():
        f = f_of[rid]
        assert st == 0 and rr <= 1e-8, rid
        u_ref, h_ref, rc = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
        assert rc == 0 and cyc == len(h_ref) - 1, (rid, f.shape)
        assert np.array_equal(u, u_ref), (rid, f.shape)


def test_server_device_fed_requests_in_a_mix(dev_ok):
    """Requests fed from device memory (right-hand side copied device to
    device at admission, solution copied into the caller's device array)
    mixed with host-fed ones: every result equals the oracle's solve."""
    import torch

    m = mg()
    sp = m.ServerParams(hbm_budget_bytes=512 << 20, max_slots=3, max_n2d=257, max_n3d=33, tol=1e-8, max_cycles=40)
    ctx = m.mg_server_create(sp)
    reqs = [(2, 129, 1, True), (3, 33, 2, False), (2, 257, 3, True), (3, 17, 4, True), (2, 65, 5, False),
            (3, 33, 6, True), (2, 129, 7, True), (2, 33, 8, False)]
    info, done = {}, {}
    pending = list(reqs)
    steps = 0
    while pending or len(done) < len(reqs):
        for _ in range(2):
            if pending:
                dim, n, seed, on_dev = pending.pop(0)
                f = inputs.uniform_rhs(dim, n, 1300 + seed)
                if on_dev:
                    fd = dev(f)
                    ud = torch.full_like(fd, float("nan"))
                    torch.cuda.synchronize()
                    rid = m.mg_server_submit_device(ctx, fd, ud)
                    info[rid] = (f, fd, ud)
                else:
                    rid = m.mg_server_submit(ctx, f)
                    info[rid] = (f, None, None)
        m.mg_server_step(ctx)
        for rid in m.mg_server_poll(ctx):
            f, fd, ud = info[rid]
            if ud is None:
                st, u, cyc, rr, _ = m.mg_server_fetch(ctx, rid, shape=f.shape)
            else:
                st, _, cyc, rr, _ = m.mg_server_fetch(ctx, rid)
                u = host(ud)
            done[rid] = (st, u, cyc, rr)
        steps += 1
        assert steps < 500
    for rid, (st, u, cyc, rr) in done.items():
        f = info[rid][0]
        assert st == 0 and rr <= 1e-8
        u_ref, h_ref, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-8, max_cycles=40)
        assert cyc == len(h_ref) - 1
        assert np.array_equal(u, u_ref)
    m.mg_destroy(ctx)
