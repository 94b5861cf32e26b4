"""The allocation-free refinement pass (mg_level_ir_update_noalloc, static
device scratch) against the allocating one (mg_level_ir_update): the same
kernels on the same inputs give the same u, r and norm, bit for bit, on two
calls in a row, the second on a smaller grid (the shared scratch keeps the
first call's contents), and launch shapes whose norm partials exceed the
scratch are rejected before anything runs."""

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def mg():
    import paper_1406_5369_amd as m

    return m


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def case(dim, n, seed):
    u = inputs.random_guess(dim, n, 40 + seed)
    e = inputs.random_guess(dim, n, 60 + seed).astype(np.float32) * np.float32(1e-3)
    f = inputs.uniform_rhs(dim, n, 80 + seed)
    k = inputs.varcoef_k(n, 90 + seed, dim=dim) if seed % 2 else None
    return u, e, f, k


def run(dim, n, seed, noalloc, **tile):
    import torch

    u, e, f, k = case(dim, n, seed)
    uo = torch.full(u.shape, -7.0, dtype=torch.float64, device="cuda")
    r = torch.full(u.shape, -7.0, dtype=torch.float32, device="cuda")
    rho = mg().mg_level_ir_update(dev(u), dev(e), dev(f), uo, r, k=dev(k) if k is not None else None,
                                  noalloc=noalloc, **tile)
    torch.cuda.synchronize()
    return uo.cpu().numpy(), r.cpu().numpy(), rho


SEQUENCES = [
    # (first call, second call on a smaller grid): dim, n, seed, tile arguments
    ((3, 65, 0, {}), (3, 33, 2, {})),
    ((3, 129, 1, dict(by=16, zchunk=8, prefetch=2, waves=8)), (3, 17, 3, dict(by=8, zchunk=2))),
    ((3, 257, 0, dict(by=16, zchunk=64, prefetch=2, waves=8, pairs=1)), (3, 65, 4, dict(pairs=1))),
    ((2, 1025, 0, dict(pairs=1)), (2, 129, 2, dict(pairs=1, zchunk=8))),
    ((2, 513, 1, dict(by=8)), (2, 33, 5, {})),
]


@pytest.mark.parametrize("first,second", SEQUENCES)
def test_noalloc_pass_equals_allocating_pass(first, second, dev_ok):
    for dim, n, seed, tile in (first, second):
        print(f"[noalloc] dim={dim} n={n} seed={seed} tile={tile}", flush=True)
        u_a, r_a, rho_a = run(dim, n, seed, False, **tile)
        u_b, r_b, rho_b = run(dim, n, seed, True, **tile)
        assert np.array_equal(u_a, u_b) and np.array_equal(r_a, r_b)
        assert rho_a == rho_b and rho_a > 0.0


def test_noalloc_rejects_shapes_beyond_its_scratch(dev_ok):
    """2D n = 8193 with 8-row tiles needs 181678 norm partials (> 131008): MG_ENOMEM,
    and the outputs are untouched."""
    import torch

    m = mg()
    n = 8193
    f = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    e = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    uo = torch.full_like(f, 3.0)
    r = torch.full_like(e, 3.0)
    with pytest.raises(m.MGError) as ei:
        m.mg_level_ir_update(u, e, f, uo, r, by=8, noalloc=True)
    assert ei.value.code == m.MG_ENOMEM
    torch.cuda.synchronize()
    assert bool((uo == 3.0).all()) and bool((r == 3.0).all())
    # the same shape through the allocating pass runs
    m.mg_level_ir_update(u, e, f, uo, r, by=8)
    torch.cuda.synchronize()
    assert not bool(uo[1:-1, 1:-1].any())
