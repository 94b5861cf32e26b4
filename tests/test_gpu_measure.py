"""Measurement hooks: the library's HIP-event brackets count only launches of
refinement steps the solve really ran (a step queued after the stop test
passed finds the stop flag set and does no work)."""

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_prof_counts_only_steps_the_solve_ran(precision, dev_ok):
    import torch

    import paper_1406_5369_amd as m

    n = 129  # 129^3 > 2^20 nodes: steps are queued four at a time
    f = inputs.uniform_rhs(3, n, 3)
    s = m.Solver(m.Params(dim=3, n=n, precision=precision))
    fd = torch.from_numpy(f).to("cuda")
    u = torch.zeros_like(fd)
    m.mg_prof_enable(s.ctx, True)
    total = 0
    for _ in range(2):
        u.zero_()
        st, cyc, hist = s.solve(u, fd, tol=1e-8, max_cycles=50)
        assert st == 0
        total += cyc
    n_sweep, ms_sweep = m.mg_prof_read(s.ctx, 0)
    n_pass, ms_pass = m.mg_prof_read(s.ctx, 1)
    m.mg_prof_enable(s.ctx, False)
    # V(2,2) plain finest-level sweeps per step (the first postsmoothing sweep
    # carries the coarse-grid correction, so the second postsmoothing sweep and):
    # in refinement steps the first presmoothing sweep starts from a zero
    # iterate, so the second presmoothing sweep, unless the two run as one
    # launch (tile family 7); in FP64 cycles the second presmoothing sweep,
    # the first one summing the norm of the previous cycle's result (tile
    # family 6: then it is the measured pass) or both, the norm a pass of its
    # own.  One refinement pass / norm pass or norm-carrying sweep per step.
    if precision == 1:
        per_step = 1 if m.mg_tile_config(s.ctx, 0, 7)[1] > 0 else 2
    else:
        per_step = 2 if m.mg_tile_config(s.ctx, 0, 6)[1] > 0 else 3
    assert n_sweep == per_step * total and n_pass == total
    assert ms_sweep > 0.0 and ms_pass > 0.0
    # reading resets the totals
    assert m.mg_prof_read(s.ctx, 0) == (0, 0.0)
    with pytest.raises(m.MGError):
        m.mg_prof_read(s.ctx, 2)
    s.close()
