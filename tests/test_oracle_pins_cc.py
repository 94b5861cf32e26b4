"""Pins of the oracle's cell-centred Neumann form (Table 1: cell-centred
discretisation, Neumann boundary, constant interpolation; the boundary of
the paper's complex-diffusion application in Section 4).

n = 2^L cells per axis, h = 1/n, cell centres at (i + 1/2) h; zero flux
through the boundary.  The pins use closed forms and constructions that share
nothing with the oracle's per-cell ghost logic:

* the cosine modes prod_a cos(k_a pi x_a) are eigenvectors of the discrete
  Neumann Laplacian with eigenvalues (4/h^2) sum_a sin^2(k_a pi h / 2), the
  constant mode (k = 0) with eigenvalue 0;
* averaging 2^d children maps a cosine mode to the coarse mode scaled by
  prod_a cos(k_a pi h / 2); constant interpolation copies the parent value;
  <P e, r>_h = 2^d <e, R r>_H;
* a red-black sweep with omega = 1 leaves a zero residual on the colour
  relaxed last (the relaxation divides by the true diagonal, boundary cells
  included);
* the multigrid solve equals the mean-zero solution of the dense matrix
  assembled from Kronecker products of the 1D Neumann second difference;
* per-cycle convergence factors of V(2,2) red-black cycles.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle

RB, JAC = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI


def cell_centres(n):
    return (np.arange(n) + 0.5) / n


def cos_mode(dim, n, kv):
    c = [np.cos(ka * np.pi * cell_centres(n)) for ka in kv]
    if dim == 2:
        return np.ascontiguousarray(np.multiply.outer(c[1], c[0]))
    return np.ascontiguousarray(np.multiply.outer(np.multiply.outer(c[2], c[1]), c[0]))


MODES = {2: [(0, 0), (1, 0), (0, 3), (2, 5), (7, 1), (15, 15)], 3: [(0, 0, 0), (1, 0, 0), (2, 3, 1), (5, 5, 7)]}


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 32), (3, 8), (3, 16)])
def test_cosine_modes_are_eigenvectors(dim, n):
    h = 1.0 / n
    for kv in MODES[dim]:
        if max(kv) >= n:
            continue
        phi = cos_mode(dim, n, kv)
        lam = (4.0 / h**2) * sum(math.sin(ka * math.pi * h / 2) ** 2 for ka in kv)
        Aphi = -oracle.cc_residual(phi, np.zeros_like(phi))
        np.testing.assert_allclose(Aphi, lam * phi, rtol=0, atol=1e-11 * max(lam, 1.0 / h**2))


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_restriction_and_interpolation_of_modes(dim, n):
    h = 1.0 / n
    for kv in MODES[dim]:
        if max(kv) >= n // 2:
            continue
        fine, coarse = cos_mode(dim, n, kv), cos_mode(dim, n // 2, kv)
        damp = np.prod([math.cos(ka * math.pi * h / 2) for ka in kv])
        np.testing.assert_allclose(oracle.cc_restrict(fine), damp * coarse, rtol=0, atol=1e-14)
    rng = np.random.default_rng(3)
    e = rng.standard_normal((n // 2,) * dim)
    up = oracle.cc_prolong_correct(np.zeros((n,) * dim), e)
    expect = e
    for ax in range(dim):
        expect = np.repeat(expect, 2, axis=ax)
    assert np.array_equal(up, expect)
    # restriction and interpolation are adjoint up to the factor 2^d
    r = rng.standard_normal((n,) * dim)
    lhs = float(np.sum(up * r))
    rhs = 2**dim * float(np.sum(e * oracle.cc_restrict(r)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8), (2, 2), (3, 2)])
def test_red_black_sweep_zeroes_the_last_colour_residual(dim, n):
    rng = np.random.default_rng(5)
    u = rng.standard_normal((n,) * dim)
    f = rng.standard_normal((n,) * dim)
    out = oracle.cc_smooth(u, f, RB, 1.0)
    r = oracle.cc_residual(out, f)
    black = (np.indices(u.shape).sum(axis=0) % 2) == 1
    assert np.abs(r[black]).max() <= 1e-12 * np.abs(r).max()
    assert np.abs(r[~black]).max() > 1e-6 * np.abs(r).max()


def test_sum_order_is_exact_on_integers():
    rng = np.random.default_rng(7)
    a = rng.integers(-1000, 1000, (16, 16, 16)).astype(np.float64)
    assert oracle.cc_sum(a) == float(a.sum())
    b = rng.standard_normal((64, 64))
    assert oracle.cc_sum(b) == pytest.approx(math.fsum(b.ravel()), rel=1e-13, abs=1e-12)


def neumann_matrix(dim, n):
    h = 1.0 / n
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    T[0, 0] = T[n - 1, n - 1] = 1.0
    T = T.tocsr() / h**2
    I = sp.identity(n)
    if dim == 2:
        return (sp.kron(I, T) + sp.kron(T, I)).toarray()
    return (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)).toarray()


@pytest.mark.parametrize("dim,n,smoother,cycle", [(2, 16, RB, 0), (2, 32, JAC, 1), (3, 8, RB, 0), (3, 8, JAC, 1),
                                                  (2, 8, RB, 2)])
def test_solve_equals_dense_mean_zero_solution(dim, n, smoother, cycle):
    rng = np.random.default_rng(11)
    f = rng.uniform(-1, 1, (n,) * dim)
    omega = 1.0 if smoother == RB else 0.8
    u, h, rc, fh = oracle.cc_solve(np.zeros_like(f), f, tol=1e-13, max_cycles=200, smoother=smoother, omega=omega,
                                   cycle=cycle)
    assert rc == 0
    A = neumann_matrix(dim, n)
    N = A.shape[0]
    # mean-zero solution: the augmented system [A 1; 1^T 0] [u; l] = [f - mean f; 0]
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    rhs = np.concatenate([f.ravel() - f.mean(), [0.0]])
    ref = np.linalg.solve(M, rhs)[:N].reshape(f.shape)
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)
    np.testing.assert_allclose(fh, f - f.mean(), rtol=0, atol=1e-14)
    assert abs(u.sum()) <= 1e-12 * np.abs(u).sum()


@pytest.mark.parametrize("dim,n", [(2, 128), (3, 32)])
def test_manufactured_cosine_solution(dim, n):
    """f = lambda phi for a cosine mode: the discrete solution is phi itself."""
    kv = (1, 2) if dim == 2 else (1, 0, 2)
    phi = cos_mode(dim, n, kv)
    h = 1.0 / n
    lam = (4.0 / h**2) * sum(math.sin(ka * math.pi * h / 2) ** 2 for ka in kv)
    u, hist, rc, _ = oracle.cc_solve(np.zeros_like(phi), lam * phi, tol=1e-12, max_cycles=60)
    assert rc == 0
    np.testing.assert_allclose(u, phi, rtol=0, atol=1e-9)


@pytest.mark.parametrize("dim,n,bound", [(2, 256, 0.1), (3, 64, 0.1)])
def test_v22_red_black_convergence_factor(dim, n, bound):
    rng = np.random.default_rng(13)
    f = rng.uniform(-1, 1, (n,) * dim)
    u, h, rc, _ = oracle.cc_solve(np.zeros_like(f), f, tol=1e-10, max_cycles=40)
    assert rc == 0
    q = [h[i + 1] / h[i] for i in range(len(h) - 1)]
    assert max(q) < bound
