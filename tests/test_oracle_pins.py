"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: discrete
eigenvalues and mode maps of the 5/7-point Laplacian and of the transfer
operators (closed forms), manufactured solutions whose discrete solution is
known exactly, a dense direct solve of a matrix assembled by a different
construction (Kronecker products / face loops), invariants (adjointness,
symmetry, order independence of a colour), and the convergence statements of
the paper (Section 4: more than 1e8 residual reduction within five V(2,2)
cycles from a random guess with f = 0).
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
import oracle

RB, JAC = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI


def mode(dim, n, kv):
    """phi_k = prod_a sin(k_a pi x_a) on the nodes of an n^dim grid (array order [k, j, i])."""
    x = inputs.node_coords(n)
    s = [np.sin(ka * np.pi * x) for ka in kv]  # s[0] along x, s[1] along y, ...
    if dim == 2:
        out = np.multiply.outer(s[1], s[0])
    else:
        out = np.multiply.outer(np.multiply.outer(s[2], s[1]), s[0])
    return np.ascontiguousarray(inputs.zero_boundary(out))


def inner(a):
    return a[(slice(1, -1),) * a.ndim]


def lam(kv, h):
    return (4.0 / h**2) * sum(math.sin(ka * math.pi * h / 2) ** 2 for ka in kv)


MODES2 = [(1, 1), (1, 2), (3, 5), (7, 2), (15, 15)]
MODES3 = [(1, 1, 1), (2, 1, 3), (5, 3, 7), (7, 7, 7)]


# ---------------------------------------------------------------- P1 operator
@pytest.mark.parametrize("dim,n,modes", [(2, 17, MODES2), (2, 33, MODES2), (3, 9, MODES3[:3]), (3, 17, MODES3)])
def test_p1_laplacian_eigenmodes(dim, n, modes):
    h = 1.0 / (n - 1)
    f0 = np.zeros((n,) * dim)
    for kv in modes:
        phi = mode(dim, n, kv)
        r = oracle.residual(phi, f0)  # = -A phi
        lk = lam(kv, h)
        np.testing.assert_allclose(inner(-r), lk * inner(phi), rtol=0, atol=1e-12 * lk)
        assert np.all(r[0] == 0) and np.all(r[-1] == 0)


@pytest.mark.parametrize("dim,n,kv", [(2, 17, (3, 2)), (3, 9, (1, 2, 3))])
def test_p1_varcoef_constant_k_scales_laplacian(dim, n, kv):
    kappa = 3.5
    h = 1.0 / (n - 1)
    phi = mode(dim, n, kv)
    k = np.full((n,) * dim, kappa)
    r = oracle.residual(phi, np.zeros_like(phi), k=k)
    lk = kappa * lam(kv, h)
    np.testing.assert_allclose(inner(-r), lk * inner(phi), rtol=0, atol=1e-12 * lk)


# ---------------------------------------------------------------- P2 Jacobi
@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
@pytest.mark.parametrize("omega", [0.8, 0.6])
def test_p2_jacobi_damps_modes_by_closed_form(dim, n, omega):
    h = 1.0 / (n - 1)
    modes = MODES2 if dim == 2 else MODES3
    for kv in modes:
        phi = mode(dim, n, kv)
        out = oracle.smooth(phi, np.zeros_like(phi), smoother=JAC, omega=omega)
        g = 1.0 - (2.0 * omega / dim) * sum(math.sin(ka * math.pi * h / 2) ** 2 for ka in kv)
        np.testing.assert_allclose(inner(out), g * inner(phi), rtol=0, atol=1e-14)


# ------------------------------------------------- Gauss-Seidel update (P11)
@pytest.mark.parametrize("dim,n", [(2, 17), (3, 9)])
@pytest.mark.parametrize("omega", [1.0, 1.3, 0.7])
@pytest.mark.parametrize("varcoef", [False, True])
def test_gs_colour_update_scales_own_residual(dim, n, omega, varcoef):
    """After relaxing one colour, that colour's residual is (1 - omega) times its old value.

    Relaxing p by omega*r_p/diag_p changes r_p by -omega*r_p and leaves the other
    nodes of the same colour untouched (they are not neighbours)."""
    rng = np.random.default_rng(7)
    u = inputs.random_guess(dim, n, 11)
    f = inputs.uniform_rhs(dim, n, 12)
    k = inputs.varcoef_k(n, 5, dim=dim) if varcoef else None
    idx = np.indices((n,) * dim).sum(axis=0) % 2
    innermask = np.zeros((n,) * dim, dtype=bool)
    innermask[(slice(1, -1),) * dim] = True
    for colour in (0, 1):
        r_old = oracle.residual(u, f, k=k)
        u1 = oracle.rbgs_colour(u, f, colour, omega=omega, k=k)
        r_new = oracle.residual(u1, f, k=k)
        m = innermask & (idx == colour)
        scale = np.abs(r_old[m]).max()
        np.testing.assert_allclose(r_new[m], (1.0 - omega) * r_old[m], rtol=0, atol=1e-11 * scale)
        # nodes of the other colour were not written
        other = (idx != colour)
        assert np.array_equal(u1[other], u[other])
        u = u1
    del rng


@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
def test_p11_colour_order_independent_and_sweep_is_red_then_black(dim, n):
    u = inputs.random_guess(dim, n, 1)
    f = inputs.uniform_rhs(dim, n, 2)
    for colour in (0, 1):
        a = oracle.rbgs_colour(u, f, colour, reverse=False)
        b = oracle.rbgs_colour(u, f, colour, reverse=True)
        assert np.array_equal(a, b)
    two = oracle.rbgs_colour(oracle.rbgs_colour(u, f, 0), f, 1)
    assert np.array_equal(two, oracle.smooth(u, f, smoother=RB, omega=1.0))


# ---------------------------------------------------------- P3 / P4 / P5
@pytest.mark.parametrize("dim,nf", [(2, 33), (3, 17)])
def test_p3_full_weighting_maps_modes(dim, nf):
    h = 1.0 / (nf - 1)
    nc = (nf - 1) // 2 + 1
    modes = MODES2[:4] if dim == 2 else MODES3[:3]
    for kv in modes:
        fc = oracle.restrict(mode(dim, nf, kv))
        expect = np.prod([math.cos(ka * math.pi * h / 2) ** 2 for ka in kv]) * mode(dim, nc, kv)
        np.testing.assert_allclose(fc, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,nf", [(2, 33), (3, 17)])
def test_p4_linear_interpolation_maps_modes(dim, nf):
    h = 1.0 / (nf - 1)
    nc = (nf - 1) // 2 + 1
    modes = MODES2[:4] if dim == 2 else MODES3[:3]
    grids = np.indices((nf,) * dim)  # grids[0] = slowest axis index
    for kv in modes:
        pe = oracle.prolong_correct(np.zeros((nf,) * dim), mode(dim, nc, kv))
        factor = np.ones((nf,) * dim)
        for a, ka in enumerate(kv):  # a = 0 is x = last array axis
            odd = (grids[dim - 1 - a] % 2) == 1
            factor = np.where(odd, factor * math.cos(ka * math.pi * h), factor)
        expect = inputs.zero_boundary(factor * mode(dim, nf, kv))
        np.testing.assert_allclose(pe, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,nf", [(2, 33), (2, 9), (3, 17), (3, 9)])
def test_p5_interpolation_is_2d_times_restriction_transpose(dim, nf):
    nc = (nf - 1) // 2 + 1
    rng = np.random.default_rng(3)
    for _ in range(3):
        e = inputs.zero_boundary(rng.standard_normal((nc,) * dim))
        r = inputs.zero_boundary(rng.standard_normal((nf,) * dim))
        lhs = float(np.sum(oracle.prolong_correct(np.zeros((nf,) * dim), e) * r))
        rhs = (2**dim) * float(np.sum(e * oracle.restrict(r)))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("dim", [2, 3])
def test_p6_coarsest_grid_solve_is_exact(dim):
    f = np.zeros((3,) * dim)
    f[(1,) * dim] = 0.7312
    u = oracle.coarsest(np.zeros_like(f), f)
    diag = (2 * dim) * 4.0  # 2d / h^2 with h = 1/2
    assert u[(1,) * dim] == pytest.approx(0.7312 / diag, rel=1e-15)
    r = oracle.residual(u, f)
    assert abs(r[(1,) * dim]) <= 4 * np.spacing(0.7312)
    if dim == 2:  # diag is a power of two: exact
        assert r[(1, 1)] == 0.0


# ---------------------------------------------------------------- P12
@pytest.mark.parametrize("dim,n,varcoef", [(2, 17, False), (3, 9, False), (2, 17, True), (3, 9, True)])
def test_p12_operator_is_symmetric(dim, n, varcoef):
    rng = np.random.default_rng(5)
    k = inputs.varcoef_k(n, 9, dim=dim) if varcoef else None
    z = np.zeros((n,) * dim)
    for _ in range(3):
        u = inputs.zero_boundary(rng.standard_normal((n,) * dim))
        v = inputs.zero_boundary(rng.standard_normal((n,) * dim))
        Au = -oracle.residual(u, z, k=k)
        Av = -oracle.residual(v, z, k=k)
        a, b = float(np.sum(Au * v)), float(np.sum(u * Av))
        assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


# ----------------------------------------------- P9 dense direct solve
def dense_poisson(dim, n):
    """-Laplace_h on inner nodes by Kronecker products of the 1D second difference."""
    m = n - 1 - 1
    h = 1.0 / (n - 1)
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h**2
    I = sp.identity(m)
    if dim == 2:  # unknown order (j, i): i fastest
        return (sp.kron(I, T) + sp.kron(T, I)).toarray()
    return (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)).toarray()


def dense_varcoef(dim, n, k):
    """-div(k grad) by a loop over faces: each face (p, q) adds k_pq/h^2 to the
    diagonal entries of its inner end nodes and -k_pq/h^2 off the diagonal."""
    m = n - 2
    h = 1.0 / (n - 1)
    N = m**dim
    A = np.zeros((N, N))

    def num(ix):  # inner node -> unknown number, None for boundary
        if any(c < 1 or c > n - 2 for c in ix):
            return None
        out = 0
        for c in reversed(ix):  # ix = (i, j[, k]); k slowest
            out = out * m + (c - 1)
        return out

    for ix in np.ndindex(*((n,) * dim)):
        for a in range(dim):
            jx = list(ix)
            jx[a] += 1
            if jx[a] > n - 1:
                continue
            kp = k[tuple(reversed(ix))]
            kq = k[tuple(reversed(jx))]
            w = 2 * kp * kq / (kp + kq) / h**2
            p, q = num(ix), num(tuple(jx))
            if p is not None:
                A[p, p] += w
            if q is not None:
                A[q, q] += w
            if p is not None and q is not None:
                A[p, q] -= w
                A[q, p] -= w
    return A


@pytest.mark.parametrize("dim,n,varcoef", [(2, 9, False), (2, 17, False), (3, 9, False), (2, 17, True), (3, 9, True)])
@pytest.mark.parametrize("smoother,omega", [(RB, 1.0), (JAC, 0.8)])
def test_p9_vcycle_solve_matches_dense_direct_solve(dim, n, varcoef, smoother, omega):
    f = inputs.uniform_rhs(dim, n, 21)
    k = inputs.varcoef_k(n, 22, dim=dim) if varcoef else None
    A = dense_varcoef(dim, n, k) if varcoef else dense_poisson(dim, n)
    x = np.linalg.solve(A, inner(f).ravel())
    u, hist, rc = oracle.solve(np.zeros_like(f), f, tol=1e-14, max_cycles=80, smoother=smoother, omega=omega, k=k)
    got = inner(u).ravel()
    assert np.linalg.norm(got - x) <= 1e-11 * np.linalg.norm(x)
    assert np.all(u[0] == 0) and np.all(u[-1] == 0)


# ----------------------------------------------- P7 / P8 manufactured
@pytest.mark.parametrize("dim,n", [(2, 129), (2, 65), (3, 33)])
def test_p7_sine_problem_discrete_solution_closed_form(dim, n):
    h = 1.0 / (n - 1)
    f = inputs.sine_rhs(dim, n)
    u, hist, rc = oracle.solve(np.zeros_like(f), f, tol=1e-13, max_cycles=40)
    amp = (math.pi**2 * h**2) / (4.0 * math.sin(math.pi * h / 2) ** 2)
    exact_discrete = amp * mode(dim, n, (1,) * dim)
    assert np.abs(u - exact_discrete).max() <= 1e-11
    cont = mode(dim, n, (1,) * dim)
    err = np.abs(u - cont).max()
    assert err == pytest.approx(amp - 1.0, rel=1e-6)
    if dim == 2 and n == 129:
        assert err == pytest.approx(5.02009e-5, rel=1e-5)


def test_p7_second_order_convergence():
    errs = []
    for n in (17, 33, 65, 129):
        f = inputs.sine_rhs(2, n)
        u, _, _ = oracle.solve(np.zeros_like(f), f, tol=1e-13, max_cycles=40)
        errs.append(np.abs(u - mode(2, n, (1, 1))).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 3.9 < r < 4.1
    assert ratios[-1] == pytest.approx(4.0, abs=2e-3)


@pytest.mark.parametrize("dim,n", [(2, 65), (3, 17)])
@pytest.mark.parametrize("smoother,omega", [(RB, 1.0), (JAC, 0.8)])
def test_p8_quadratic_solution_reproduced_exactly(dim, n, smoother, omega):
    uex, f = inputs.quadratic_problem(dim, n)
    u, _, _ = oracle.solve(np.zeros_like(f), f, tol=1e-14, max_cycles=60, smoother=smoother, omega=omega)
    assert np.abs(u - inputs.zero_boundary(uex.copy())).max() <= 1e-13


# ----------------------------------------------- P10 / paper convergence
@pytest.mark.parametrize("dim,n", [(2, 129), (2, 257), (3, 33), (3, 65)])
def test_p10_vcycle_convergence_factor_rbgs(dim, n):
    f = inputs.uniform_rhs(dim, n, 31)
    u, hist, _ = oracle.solve(np.zeros_like(f), f, tol=1e-10, max_cycles=30)
    q = hist[1:] / hist[:-1]
    assert np.all(q < 0.15), q


@pytest.mark.parametrize("dim,n", [(2, 257), (3, 33)])
def test_p10_vcycle_convergence_factor_jacobi(dim, n):
    f = inputs.uniform_rhs(dim, n, 32)
    u, hist, _ = oracle.solve(np.zeros_like(f), f, tol=1e-10, max_cycles=40, smoother=JAC, omega=0.8)
    q = hist[1:] / hist[:-1]
    assert np.all(q < 0.35), q


@pytest.mark.parametrize("n", [513, 1025])
def test_paper_five_cycles_reduce_residual_1e8_from_random_guess(n):
    """Section 4: with f = 0 and a random initial guess (Section 2.1), five V(2,2)
    cycles reduce the L2 residual by more than 1e8.  Gated for the 2D RBGS
    solver, where it reproduces; the paper leaves the random distribution
    unspecified, and with U[-1, 1] the 3D RBGS and the Jacobi solvers reach
    about 1.5e7 and 1e4-1e5 (recorded, not gated)."""
    u0 = inputs.random_guess(2, n, 41)
    f = np.zeros_like(u0)
    _, hist, _ = oracle.solve(u0, f, tol=0.0, max_cycles=5, smoother=RB, omega=1.0)
    assert len(hist) == 6
    assert hist[0] / hist[5] > 1e8


def test_varcoef_solver_converges():
    n = 33
    k = inputs.varcoef_k(n, 1)
    f = inputs.uniform_rhs(3, n, 2)
    _, hist, rc = oracle.solve(np.zeros_like(f), f, tol=1e-8, max_cycles=40, k=k)
    assert rc == 0
    q = hist[1:] / hist[:-1]
    assert np.all(q < 0.3), q


# ----------------------------------------------- single precision forms
@pytest.mark.parametrize("dim,n", [(2, 65), (3, 17)])
def test_fp32_cycle_tracks_fp64_cycle(dim, n):
    f = inputs.uniform_rhs(dim, n, 51)
    u64 = oracle.vcycle(np.zeros_like(f), f)
    u32 = oracle.vcycle(np.zeros(f.shape, np.float32), f.astype(np.float32))
    assert np.linalg.norm(u32 - u64) <= 1e-5 * np.linalg.norm(u64)


@pytest.mark.parametrize("dim,n,varcoef", [(2, 129, False), (3, 33, False), (3, 17, True)])
def test_mixed_precision_refinement_reaches_fp64_solution(dim, n, varcoef):
    f = inputs.uniform_rhs(dim, n, 61)
    k = inputs.varcoef_k(n, 62, dim=dim) if varcoef else None
    u64, h64, _ = oracle.solve(np.zeros_like(f), f, tol=1e-13, max_cycles=60, k=k)
    uir, hir, _ = oracle.solve_ir_f32(np.zeros_like(f), f, tol=1e-13, max_cycles=60, k=k)
    assert hir[-1] <= 1e-12 * hir[0] or len(hir) == 61
    assert np.linalg.norm(uir - u64) <= 1e-10 * np.linalg.norm(u64)
    # refinement reaches 1e-8 in a similar number of steps as the FP64 solve
    n64 = int(np.argmax(h64 <= 1e-8 * h64[0]))
    nir = int(np.argmax(hir <= 1e-8 * hir[0]))
    assert nir <= n64 + 2


# ------------------------------------------------ residual norm (Section 2.4 Application, L2 residual)
@pytest.mark.parametrize("dim,n,modes", [(2, 17, MODES2), (2, 33, MODES2[:3]), (3, 9, MODES3[:3]), (3, 17, MODES3)])
def test_norm_of_eigenmode_residual_closed_form(dim, n, modes):
    """With f = 0 and u = phi_k the residual is -lambda_k phi_k; over the inner
    nodes sum_i sin^2(k pi i h) = (n-1)/2 for every axis, so the unscaled
    Euclidean norm is lambda_k ((n-1)/2)^(d/2) (closed form)."""
    h = 1.0 / (n - 1)
    f0 = np.zeros((n,) * dim)
    for kv in modes:
        phi = mode(dim, n, kv)
        got = oracle.residual_norm(phi, f0)
        want = lam(kv, h) * ((n - 1) / 2.0) ** (dim / 2.0)
        assert got == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 17), (2, 65), (3, 5), (3, 9), (3, 33)])
@pytest.mark.parametrize("varcoef", [False, True])
def test_norm_is_euclidean_norm_of_pinned_residual(dim, n, varcoef):
    """The norm is the 2-norm of the residual array (itself pinned by P1, P9
    and P12) over every inner node: compared with numpy's Euclidean norm,
    random u and f, Laplacian and variable coefficients."""
    rng = np.random.default_rng(40 + n + dim)
    k = inputs.varcoef_k(n, 41, dim=dim) if varcoef else None
    for _ in range(2):
        u = inputs.zero_boundary(rng.uniform(-1, 1, (n,) * dim))
        f = inputs.zero_boundary(rng.uniform(-1, 1, (n,) * dim))
        r = oracle.residual(u, f, k=k)
        want = float(np.linalg.norm(r.ravel()))
        assert oracle.residual_norm(u, f, k=k) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 9)])
def test_norm_counts_every_inner_node_once(dim, n):
    """A residual of 3 at one inner node has norm 3, wherever the node is
    (corners, edges and faces of the inner region included)."""
    u = np.zeros((n,) * dim)
    for ix in [(1,) * dim, (n - 2,) * dim, (1,) + (n - 2,) * (dim - 1), (n - 2,) + (1,) * (dim - 1),
               (n // 2,) * dim]:
        f = np.zeros((n,) * dim)
        f[ix] = 3.0
        assert oracle.residual_norm(u, f) == 3.0
    f = inputs.zero_boundary(np.ones((n,) * dim))
    assert oracle.residual_norm(u, f) == pytest.approx(math.sqrt((n - 2) ** dim), rel=1e-15)
