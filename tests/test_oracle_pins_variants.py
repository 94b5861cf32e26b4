"""Pins of the oracle's cycle and smoother variants (Algorithm 1's "direct
solver or CG" coarsest solve, the W- and F-cycles of the recursion with
gamma > 1, the symmetric red-black smoother of Table 1's "red-black
variants") against formulations that share no code with it:

* the multigrid error-propagation operator assembled from dense matrices
  (Kronecker products of the 1D second difference and of the 1D
  full-weighting stencil, P = 2^d R^T, colour relaxations as dense
  operators) by the textbook recursion M_l = S_post (I - P (I - M_{l+1}^g)
  A_{l+1}^{-1} R A_l) S_pre, compared with one cycle of the oracle on a
  random error (f = 0);
* conjugate gradients against the dense direct solve (exact after as many
  steps as unknowns) and against the Krylov-subspace minimiser of the energy
  norm after k steps;
* the A-self-adjointness of the cycle with symmetric smoothing.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
import oracle

RB, JAC, SYM = oracle.SMOOTH_RBGS, oracle.SMOOTH_JACOBI, oracle.SMOOTH_RBGS_SYM
V, W, F = oracle.CYCLE_V, oracle.CYCLE_W, oracle.CYCLE_F


def inner(a):
    return a[(slice(1, -1),) * a.ndim]


def embed(x, dim, n):
    out = np.zeros((n,) * dim)
    out[(slice(1, -1),) * dim] = x.reshape((n - 2,) * dim)
    return out


def lap1(n):
    m, h = n - 2, 1.0 / (n - 1)
    return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h**2


def kron_sum(dim, T):
    I = sp.identity(T.shape[0])
    if dim == 2:  # unknown order (j, i): i fastest
        return (sp.kron(I, T) + sp.kron(T, I)).toarray()
    return (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)).toarray()


def fw1(nf):
    """1D full weighting (1/4, 1/2, 1/4) from fine inner nodes to coarse inner nodes."""
    nc = (nf - 1) // 2 + 1
    R = np.zeros((nc - 2, nf - 2))
    for I in range(1, nc - 1):
        for d, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            R[I - 1, 2 * I + d - 1] = w
    return R


def kron_pow(M, dim):
    out = M
    for _ in range(dim - 1):
        out = np.kron(out, M)
    return out


def colour_mask(dim, n, colour):
    idx = np.indices((n - 2,) * dim).sum(axis=0) + dim  # inner node (i, j[, k]) sums, 1-based
    return ((idx % 2) == colour).ravel().astype(float)


def smoother_ops(A, dim, n, smoother, omega):
    """Error operators of one pre- and one post-smoothing sweep."""
    Dinv = np.diag(1.0 / np.diag(A))
    I = np.eye(A.shape[0])
    if smoother == JAC:
        S = I - omega * Dinv @ A
        return S, S
    Er = I - omega * np.diag(colour_mask(dim, n, 0)) @ Dinv @ A
    Eb = I - omega * np.diag(colour_mask(dim, n, 1)) @ Dinv @ A
    pre = Eb @ Er  # red, then black
    post = Er @ Eb if smoother == SYM else pre
    return pre, post


def cycle_operator(dim, n, smoother, omega, nu1, nu2, kind):
    """Dense error-propagation operator of one cycle (Laplacian, exact solve on n = 3)."""
    ns = []
    m = n
    while True:
        ns.append(m)
        if m == 3:
            break
        m = (m - 1) // 2 + 1
    A = [kron_sum(dim, lap1(m)) for m in ns]

    def M(l, kind):
        if l == len(ns) - 1:
            return np.zeros_like(A[l])  # exact solve kills the error
        R = kron_pow(fw1(ns[l]), dim)
        P = (2**dim) * R.T
        pre, post = smoother_ops(A[l], dim, ns[l], smoother, omega)
        if kind == V:
            coarse_err = M(l + 1, V)
        elif kind == W:
            Mc = M(l + 1, W)
            coarse_err = Mc @ Mc
        else:
            coarse_err = M(l + 1, V) @ M(l + 1, F)
        I_c = np.eye(A[l + 1].shape[0])
        cgc = np.eye(A[l].shape[0]) - P @ (I_c - coarse_err) @ np.linalg.solve(A[l + 1], R @ A[l])
        return np.linalg.matrix_power(post, nu2) @ cgc @ np.linalg.matrix_power(pre, nu1)

    return M(0, kind)


@pytest.mark.parametrize("dim,n", [(2, 9), (2, 17), (3, 9)])
@pytest.mark.parametrize("kind", [V, W, F])
@pytest.mark.parametrize("smoother,omega,nu", [(RB, 1.0, (2, 2)), (SYM, 1.0, (2, 1)), (JAC, 0.8, (1, 2))])
def test_cycle_equals_dense_error_operator(dim, n, kind, smoother, omega, nu):
    M = cycle_operator(dim, n, smoother, omega, nu[0], nu[1], kind)
    e0 = inner(inputs.random_guess(dim, n, 31)).ravel()
    got = oracle.vcycle(embed(e0, dim, n), np.zeros((n,) * dim), smoother=smoother, omega=omega, nu1=nu[0],
                        nu2=nu[1], cycle=kind)
    expect = M @ e0
    assert np.linalg.norm(inner(got).ravel() - expect) <= 1e-12 * np.linalg.norm(e0)


@pytest.mark.parametrize("kind", [V, W, F])
def test_variants_differ_where_they_should(kind):
    """The W- and F-cycles differ from the V-cycle from three levels on, the
    symmetric smoother from the plain one (else the pins above could not tell
    them apart)."""
    dim, n = 2, 17
    e0 = inputs.random_guess(dim, n, 32)
    z = np.zeros_like(e0)
    a = oracle.vcycle(e0, z, cycle=kind)
    b = oracle.vcycle(e0, z, cycle=V)
    assert (kind == V) == np.array_equal(a, b)
    c = oracle.vcycle(e0, z, smoother=SYM, cycle=kind)
    assert not np.array_equal(a, c)


@pytest.mark.parametrize("dim,n", [(2, 17), (3, 9)])
@pytest.mark.parametrize("kind", [V, W])
def test_symmetric_smoothing_gives_self_adjoint_cycle(dim, n, kind):
    """With the post-smoother the A-adjoint of the pre-smoother (black-red after
    red-black, nu1 = nu2) and P = 2^d R^T, the cycle's error operator M is
    self-adjoint in the energy inner product: <A M x, y> = <A x, M y>."""
    A = kron_sum(dim, lap1(n))
    x = inner(inputs.random_guess(dim, n, 33)).ravel()
    y = inner(inputs.random_guess(dim, n, 34)).ravel()
    z = np.zeros((n,) * dim)

    def M(v, sm):
        return inner(oracle.vcycle(embed(v, dim, n), z, smoother=sm, cycle=kind)).ravel()

    lhs, rhs = (A @ M(x, SYM)) @ y, (A @ x) @ M(y, SYM)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-14 * np.linalg.norm(A @ x) * np.linalg.norm(y)
    # red-first post-smoothing breaks the symmetry
    lhs, rhs = (A @ M(x, RB)) @ y, (A @ x) @ M(y, RB)
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


@pytest.mark.parametrize("dim,n,iters", [(2, 5, 9), (2, 9, 60), (3, 5, 27), (3, 9, 120)])
def test_cg_coarsest_solve_reaches_dense_solution(dim, n, iters):
    f = inputs.uniform_rhs(dim, n, 35)
    x = np.linalg.solve(kron_sum(dim, lap1(n)), inner(f).ravel())
    got = inner(oracle.coarsest_cg(np.zeros_like(f), f, iters=iters)).ravel()
    assert np.linalg.norm(got - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 9)])
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cg_iterate_minimises_energy_error_over_krylov_space(dim, n, k):
    """After k steps from zero, CG's iterate is the A-norm-closest point of
    span{f, A f, ..., A^(k-1) f} to the solution: x_k = V (V^T A V)^-1 V^T f."""
    f = inputs.uniform_rhs(dim, n, 36)
    A = kron_sum(dim, lap1(n))
    b = inner(f).ravel()
    Kb = [b]
    for _ in range(k - 1):
        Kb.append(A @ Kb[-1])
    Q, _ = np.linalg.qr(np.array(Kb).T)
    xk = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
    got = inner(oracle.coarsest_cg(np.zeros_like(f), f, iters=k)).ravel()
    assert np.linalg.norm(got - xk) <= 1e-9 * np.linalg.norm(xk)


def test_cg_coarsest_solve_with_one_unknown_is_exact():
    """At n = 3 one CG step is the exact solve u = f / diag."""
    for dim in (2, 3):
        f = np.zeros((3,) * dim)
        f[(1,) * dim] = 5.0
        u = oracle.coarsest_cg(np.zeros_like(f), f, iters=1)
        assert u[(1,) * dim] == pytest.approx(5.0 / (2 * dim * 4.0), rel=1e-15)


@pytest.mark.parametrize("dim,n,coarse_n", [(2, 33, 5), (2, 33, 9), (3, 17, 5), (3, 17, 9)])
@pytest.mark.parametrize("kind", [V, W, F])
def test_solve_with_cg_coarsest_matches_dense_direct_solve(dim, n, coarse_n, kind):
    f = inputs.uniform_rhs(dim, n, 37)
    x = np.linalg.solve(kron_sum(dim, lap1(n)), inner(f).ravel()) if n ** dim <= 40000 else None
    u, hist, rc = oracle.solve(np.zeros_like(f), f, tol=1e-13, max_cycles=60, cycle=kind, coarse_n=coarse_n)
    assert rc == 0
    q = np.array(hist[1:]) / np.array(hist[:-1])
    assert q[hist[1:] >= 1e-10 * hist[0]].max() < 0.15
    if x is not None:
        assert np.linalg.norm(inner(u).ravel() - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("dim,n", [(2, 65), (3, 33)])
def test_w_and_f_cycles_contract_at_least_as_well_as_v(dim, n):
    """Per-cycle residual reduction: W <= F <= V (up to 10 %) on Poisson with RBGS V(2,2)."""
    f = inputs.uniform_rhs(dim, n, 38)

    def rate(kind):
        _, h, _ = oracle.solve(np.zeros_like(f), f, tol=1e-10, max_cycles=30, cycle=kind)
        return (h[-1] / h[0]) ** (1.0 / (len(h) - 1))

    rv, rf, rw = rate(V), rate(F), rate(W)
    assert rw <= rf * 1.1 and rf <= rv * 1.1
