"""Pins of the oracle's constant-stencil operator (Section 2.2: a stencil with
constant entries declared for the discretisation; the Laplacian's 5-/7-point
stencil is one instance).  A = (1/h^2) stencil, coefficients centre first,
then -x, +x, -y, +y[, -z, +z], the same stencil with each level's h.

None of these retypes the oracle's per-node expression:

* symmetric stencils: sine modes are eigenvectors with the closed-form
  eigenvalue c (s0 - 2a cos(kx pi h) - 2b cos(ky pi h) [- 2g cos(kz pi h)]);
* any stencil: the residual equals the one of a sparse matrix assembled from
  Kronecker products of 1D shift matrices;
* the smoother: after a red-black sweep with omega = 1 the residual vanishes
  on black nodes (pins the diagonal c s0); a Jacobi sweep scales an eigenmode
  by 1 - omega lambda / (c s0);
* the coarsest solve zeroes the residual of the single unknown;
* the multigrid solve (V, W, F; RBGS, symmetric RBGS, Jacobi) equals the dense
  direct solve of the assembled matrix;
* the Laplacian's stencil reproduces the Laplacian path bit for bit.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
import oracle

RB, JAC, SYM = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI, oracle.SMOOTH_RBGS_SYM

# operator-level pins take any stencil: symmetric with a diagonal shift, and
# non-symmetric (convection-like) ones
ANISO2 = [4.0, -1.0, -1.0, -0.6, -0.6]
ANISO3 = [5.0, -1.0, -1.0, -0.7, -0.7, -0.4, -0.4]
SKEW2 = [4.4, -1.3, -0.7, -1.1, -0.9]
SKEW3 = [6.5, -1.2, -0.8, -1.15, -0.85, -1.3, -0.7]
# Solves need a stencil that re-discretises consistently with each level's
# h: a second-order operator, entries summing to zero (anisotropic diffusion;
# a mildly skewed 3D one converges too).  A diagonal shift is a reaction term
# that the 1/h^2 scaling changes by 4 per level, and the coarse correction
# then diverges.
ZSUM2 = [3.2, -1.0, -1.0, -0.6, -0.6]
ZSUM3 = [4.2, -1.0, -1.0, -0.7, -0.7, -0.4, -0.4]
ZSKEW3 = [6.0, -1.2, -0.8, -1.1, -0.9, -1.05, -0.95]


def stencil_matrix(dim, n, st):
    """(1/h^2) stencil on the inner nodes, assembled from 1D shift matrices
    (x fastest: the x operator is the last Kronecker factor)."""
    m = n - 2
    c = float(n - 1) ** 2
    eye = sp.identity(m, format="csr")
    lo, hi = sp.eye(m, k=-1, format="csr"), sp.eye(m, k=1, format="csr")  # (lo u)_i = u_{i-1}

    def axis(op, a):  # op acting along axis a (0 = x)
        mats = [eye] * dim
        mats[dim - 1 - a] = op
        out = mats[0]
        for mm in mats[1:]:
            out = sp.kron(out, mm, format="csr")
        return out

    A = st[0] * sp.identity(m**dim, format="csr")
    for a in range(dim):
        A = A + st[1 + 2 * a] * axis(lo, a) + st[2 + 2 * a] * axis(hi, a)
    return c * A


def inner(a):
    return a[(slice(1, -1),) * a.ndim]


def sine_mode(dim, n, kv):
    x = inputs.node_coords(n)
    s = [np.sin(k * np.pi * x) for k in kv]
    if dim == 2:
        return np.ascontiguousarray(np.multiply.outer(s[1], s[0]))
    return np.ascontiguousarray(np.multiply.outer(np.multiply.outer(s[2], s[1]), s[0]))


@pytest.mark.parametrize("dim,n,st", [(2, 33, ANISO2), (3, 17, ANISO3)])
@pytest.mark.parametrize("kv", [(1, 1, 1), (3, 5, 2), (7, 2, 6)])
def test_symmetric_stencil_sine_eigenvalues(dim, n, st, kv):
    kv = kv[:dim]
    phi = inputs.zero_boundary(sine_mode(dim, n, kv))
    h = 1.0 / (n - 1)
    lam = st[0] + sum(2.0 * st[1 + 2 * a] * np.cos(kv[a] * np.pi * h) for a in range(dim))
    lam *= 1.0 / h**2
    r = oracle.st_residual(phi, np.zeros_like(phi), st)
    np.testing.assert_allclose(r, -lam * phi, rtol=0, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("dim,n,st", [(2, 17, SKEW2), (2, 33, ANISO2), (3, 9, SKEW3), (3, 17, ANISO3)])
def test_residual_equals_assembled_matrix(dim, n, st):
    u = inputs.zero_boundary(inputs.random_guess(dim, n, 3))
    f = inputs.uniform_rhs(dim, n, 4)
    A = stencil_matrix(dim, n, st)
    expect = inner(f).ravel() - A @ inner(u).ravel()
    r = oracle.st_residual(u, f, st)
    np.testing.assert_allclose(inner(r).ravel(), expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
    assert not np.any(r[0]) and not np.any(r[-1])


@pytest.mark.parametrize("dim,n,st", [(2, 33, SKEW2), (3, 17, SKEW3)])
def test_rbgs_sweep_zeroes_black_residual(dim, n, st):
    u = inputs.zero_boundary(inputs.random_guess(dim, n, 5))
    f = inputs.uniform_rhs(dim, n, 6)
    out = oracle.st_smooth(u, f, st, RB, 1.0)
    r = inner(oracle.st_residual(out, f, st))
    idx = np.indices(r.shape).sum(axis=0) + dim  # parity of i + j [+ k] on the full grid
    black = (idx & 1) == 1
    scale = np.abs(inner(oracle.st_residual(u, f, st))).max()
    assert np.abs(r[black]).max() <= 1e-12 * scale
    assert np.abs(r[~black]).max() > 1e-3 * scale  # red residuals are not zero after the black half
    # black first (the symmetric smoother's post-smoothing sweep): red residuals vanish
    out2 = oracle.st_smooth(u, f, st, SYM, 1.0)
    r2 = inner(oracle.st_residual(out2, f, st))
    assert np.abs(r2[~black]).max() <= 1e-12 * scale


@pytest.mark.parametrize("dim,n,st", [(2, 33, ANISO2), (3, 17, ANISO3)])
def test_jacobi_scales_eigenmode(dim, n, st):
    kv = (2, 3, 1)[:dim]
    phi = inputs.zero_boundary(sine_mode(dim, n, kv))
    h = 1.0 / (n - 1)
    lam = (st[0] + sum(2.0 * st[1 + 2 * a] * np.cos(kv[a] * np.pi * h) for a in range(dim))) / h**2
    omega = 0.8
    out = oracle.st_smooth(phi, np.zeros_like(phi), st, JAC, omega)
    factor = 1.0 - omega * lam * h**2 / st[0]
    np.testing.assert_allclose(out, factor * phi, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim,st", [(2, SKEW2), (3, SKEW3)])
def test_coarsest_solve_exact(dim, st):
    f = np.zeros((3,) * dim)
    f[(1,) * dim] = 2.5
    u = oracle.st_coarsest(f, st)
    r = oracle.st_residual(u, f, st)
    assert abs(r[(1,) * dim]) <= 1e-15 * 2.5
    assert u[(1,) * dim] == pytest.approx(2.5 / (4.0 * st[0]))


@pytest.mark.parametrize("dim,n,st", [(2, 33, ZSUM2), (3, 9, ZSKEW3), (3, 17, ZSUM3)])
@pytest.mark.parametrize("smoother,cycle", [(RB, 0), (SYM, 0), (JAC, 0), (RB, 1), (RB, 2)])
def test_solve_equals_dense_solve(dim, n, st, smoother, cycle):
    f = inputs.uniform_rhs(dim, n, 7)
    omega = 0.8 if smoother == JAC else 1.0
    u, hist, rc = oracle.st_solve(np.zeros_like(f), f, st, tol=1e-12, max_cycles=200, smoother=smoother, omega=omega,
                                  cycle=cycle)
    assert rc == 0
    A = stencil_matrix(dim, n, st).toarray()
    x = np.linalg.solve(A, inner(f).ravel())
    np.testing.assert_allclose(inner(u).ravel(), x, rtol=0, atol=1e-9 * np.abs(x).max())
    q = [hist[i + 1] / hist[i] for i in range(min(4, len(hist) - 1))]
    assert max(q) < (0.7 if smoother == JAC else 0.4)


@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
@pytest.mark.parametrize("smoother", [RB, JAC, SYM])
def test_laplacian_stencil_reproduces_laplacian_path(dim, n, smoother):
    lap = [2.0 * dim] + [-1.0] * (2 * dim)
    f = inputs.uniform_rhs(dim, n, 8)
    omega = 0.8 if smoother == JAC else 1.0
    u1, h1, _ = oracle.st_solve(np.zeros_like(f), f, lap, tol=1e-10, max_cycles=20, smoother=smoother, omega=omega)
    u2, h2, _ = oracle.solve(np.zeros_like(f), f, tol=1e-10, max_cycles=20, smoother=smoother, omega=omega)
    assert np.array_equal(u1, u2) and np.array_equal(h1, h2)
