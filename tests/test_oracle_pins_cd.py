"""Pins of the oracle's complex-diffusion form (Section 4, Eq. (2) with the
complex diffusivity g(Im u) = e^{i theta} / (1 + (Im u / (k theta))^2),
homogeneous Neumann boundary, averaged finite differences on a cell-centred
grid, implicit Euler in time, FAS with lagged diffusivity per time step).

The pins share no code with the oracle's per-cell complex arithmetic:

* g against numpy's complex arithmetic on the definition;
* the operator N(u) = u / tau - div(g grad u) against a sparse matrix
  assembled face by face from g(u) (face coefficient = mean of the two
  cells' g);
* with a constant diffusivity (k theta huge): cosine modes are eigenvectors
  with eigenvalue 1/tau + e^{i theta} lambda_k, the FAS solve equals numpy's
  dense complex solve, and with theta -> 0 one time step maps a cosine mode
  to phi / (1 + tau lambda_k) (the heat equation);
* the nonlinear solve satisfies the independently assembled system, and a
  time step conserves the complex mass sum u (zero flux through the
  boundary) up to tau sum r;
* FAS convergence: the paper's 1e5 residual reduction within five V(2,2)
  cycles, and per-cycle factors.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import inputs
import oracle

RB, JAC = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI


def cos_mode(dim, n, kv):
    c = [np.cos(ka * np.pi * inputs.cell_centres(n)) for ka in kv]
    if dim == 2:
        return np.ascontiguousarray(np.multiply.outer(c[1], c[0]))
    return np.ascontiguousarray(np.multiply.outer(np.multiply.outer(c[2], c[1]), c[0]))


def matrix_of(u, P, dim, n):
    """Sparse matrix of v -> v / tau - div(g grad v) with g = g(Im u) frozen."""
    g = np.exp(1j * P.theta) / (1.0 + (u.imag / (P.k * P.theta)) ** 2)
    c = float(n) ** 2
    N = u.size
    gf = g.ravel()
    rows, cols, vals = [], [], []
    diag = np.full(N, 1.0 / P.tau, dtype=complex)
    strides = [1, n, n * n][:dim]
    idx = np.arange(N).reshape((n,) * dim)
    for ax, st in enumerate(strides):
        axis = dim - 1 - ax  # numpy axis of this stride (x is the last axis)
        lo = np.take(idx, np.arange(n - 1), axis=axis).ravel()
        hi = lo + st
        gface = 0.5 * (gf[lo] + gf[hi])
        for a, b in ((lo, hi), (hi, lo)):
            rows.append(a)
            cols.append(b)
            vals.append(-c * gface)
            np.add.at(diag, a, c * gface)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def test_diffusivity_matches_definition():
    P = oracle.CD(tau=1e-3, k=0.1)
    u = inputs.random_complex(2, 32, 1, 0.05)
    g = oracle.cd_g(u, P)
    ref = np.exp(1j * P.theta) / (1.0 + (u.imag / (P.k * P.theta)) ** 2)
    np.testing.assert_allclose(g, ref, rtol=2e-16 * 8, atol=0)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_operator_equals_face_assembled_matrix(dim, n):
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u = inputs.random_complex(dim, n, 2, 0.05)
    M = matrix_of(u, P, dim, n)
    got = oracle.cd_apply(u, P).ravel()
    ref = M @ u.ravel()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_constant_diffusivity_cosine_eigenmodes(dim, n):
    P = oracle.CD(tau=10.0 / n**2, theta=math.pi / 30, k=1e300)  # k theta huge: g = e^{i theta}
    h = 1.0 / n
    for kv in ([(1, 0), (3, 2), (7, 7)] if dim == 2 else [(1, 0, 0), (2, 1, 3)]):
        phi = cos_mode(dim, n, kv).astype(np.complex128)
        lam = (4.0 / h**2) * sum(math.sin(ka * math.pi * h / 2) ** 2 for ka in kv)
        mu = 1.0 / P.tau + np.exp(1j * P.theta) * lam
        np.testing.assert_allclose(oracle.cd_apply(phi, P), mu * phi, rtol=0, atol=1e-11 * abs(mu))


@pytest.mark.parametrize("dim,n,smoother", [(2, 16, RB), (3, 8, RB), (2, 16, JAC)])
def test_linear_fas_solve_equals_dense_solve(dim, n, smoother):
    P = oracle.CD(tau=100.0 / n**2, k=1e300)
    f = inputs.random_complex(dim, n, 3)
    u = np.zeros_like(f)
    omega = 1.0 if smoother == RB else 0.8
    for _ in range(60):
        u = oracle.cd_fas(u, f, P, smoother=smoother, omega=omega)
    M = matrix_of(np.zeros_like(f), P, dim, n)
    ref = spla.spsolve(M.tocsc(), f.ravel()).reshape(f.shape)
    assert np.linalg.norm(u - ref) <= 1e-11 * np.linalg.norm(ref)


def test_heat_limit_one_time_step():
    """theta -> 0 with k theta fixed and huge: g = 1, one implicit Euler step
    maps a cosine mode phi to phi / (1 + tau lambda)."""
    dim, n = 2, 64
    P = oracle.CD(tau=20.0 / n**2, theta=1e-300, k=1e300 / 1e-300 * 1e-300)
    P.k = 1e300 / P.theta  # k theta = 1e300
    phi = cos_mode(dim, n, (2, 3)).astype(np.complex128)
    h = 1.0 / n
    lam = (4.0 / h**2) * (math.sin(2 * math.pi * h / 2) ** 2 + math.sin(3 * math.pi * h / 2) ** 2)
    u, cyc, hist, rc = oracle.cd_run(phi, P, steps=1, tol=1e-13, max_cycles=40)
    assert rc == 0
    np.testing.assert_allclose(u, phi / (1.0 + P.tau * lam), rtol=0, atol=1e-11)


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_nonlinear_step_solves_assembled_system_and_conserves_mass(dim, n):
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 4)
    u1, cyc, hist, rc = oracle.cd_run(u0, P, steps=1, tol=1e-12, max_cycles=60)
    assert rc == 0
    f = u0 / P.tau
    M = matrix_of(u1, P, dim, n)
    res = f.ravel() - M @ u1.ravel()
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(f)
    assert abs(u1.sum() - u0.sum()) <= 1e-9 * np.abs(u0).sum()
    assert np.abs(u1.imag).max() > 1e-4  # the complex diffusivity makes an imaginary part


@pytest.mark.parametrize("dim,n", [(2, 128), (3, 32)])
def test_fas_reduces_residual_by_1e5_within_five_cycles(dim, n):
    """Section 4: for complex diffusion the residual is reduced by 1e5 (within
    the five V(2,2) cycles of its Poisson statement)."""
    P = oracle.CD(tau=10.0 / n**2, k=0.1)
    u0 = inputs.noisy_image(dim, n, 5)
    u, cyc, hist, rc = oracle.cd_run(u0, P, steps=3, tol=1e-5, max_cycles=5)
    assert rc == 0 and all(c <= 5 for c in cyc)
    for h in hist:
        q = [h[i + 1] / h[i] for i in range(len(h) - 1)]
        assert max(q) < 0.15
