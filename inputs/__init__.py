"""Seeded synthetic inputs for the multigrid solver.

This module only draws and lays out input data: right-hand sides, initial
guesses, coefficient fields, grid-size lists and request arrival times.  It
holds none of the solver's arithmetic, so the plain CPU reference in
``oracle/`` and the HIP library in ``paper_1406_5369_amd/`` can both consume
exactly the same arrays without sharing any method code.

Layout convention (shared by every consumer): a node-based grid with ``n``
nodes per axis, boundary nodes included, stored as a C-ordered float64 array
of shape ``(n, n)`` (index ``[j, i]``) or ``(n, n, n)`` (index ``[k, j, i]``),
x fastest.  Node ``i`` sits at ``x = i / (n - 1)`` on the unit square / cube.
Boundary entries of right-hand sides and initial guesses are zero.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "check_edge",
    "node_coords",
    "zero_boundary",
    "sine_rhs",
    "quadratic_problem",
    "uniform_rhs",
    "random_guess",
    "varcoef_k",
    "batch_problem",
    "serving_requests",
    "Request",
    "cell_centres",
    "random_cells",
    "noisy_image",
    "random_complex",
]


def check_edge(n: int) -> int:
    """Return L for an edge of n = 2**L + 1 nodes (L >= 1), else raise."""
    if n < 3 or ((n - 1) & (n - 2)) != 0:
        raise ValueError(f"grid edge must be 2**L+1 with L>=1, got {n}")
    return int(round(math.log2(n - 1)))


def node_coords(n: int) -> np.ndarray:
    """Node coordinates 0, h, ..., 1 with h = 1/(n-1)."""
    return np.arange(n, dtype=np.float64) / float(n - 1)


def zero_boundary(a: np.ndarray) -> np.ndarray:
    """Set every boundary node of a 2D/3D node array to zero (in place)."""
    for ax in range(a.ndim):
        sl = [slice(None)] * a.ndim
        sl[ax] = 0
        a[tuple(sl)] = 0.0
        sl[ax] = -1
        a[tuple(sl)] = 0.0
    return a


def sine_rhs(dim: int, n: int) -> np.ndarray:
    """Right-hand side d*pi^2 * prod_a sin(pi x_a) of the smooth test problem.

    With -Laplace(u) = f and zero Dirichlet data the continuous solution is
    u = prod_a sin(pi x_a) (the 2D case is the 129 x 129 workload).
    """
    check_edge(n)
    s = np.sin(np.pi * node_coords(n))
    s[0] = 0.0
    s[-1] = 0.0
    if dim == 2:
        f = (2.0 * np.pi**2) * np.multiply.outer(s, s)
    elif dim == 3:
        f = (3.0 * np.pi**2) * np.multiply.outer(np.multiply.outer(s, s), s)
    else:
        raise ValueError("dim must be 2 or 3")
    return np.ascontiguousarray(zero_boundary(f))


def quadratic_problem(dim: int, n: int) -> tuple[np.ndarray, np.ndarray]:
    """(u, f) for u = prod_a x_a (1 - x_a), f = -Laplace(u).

    Returns the nodal values of the continuous solution and right-hand side.
    """
    check_edge(n)
    x = node_coords(n)
    q = x * (1.0 - x)
    if dim == 2:
        u = np.multiply.outer(q, q)
        # -d2/dx2 of q(x) is 2, so -Laplace(q(x)q(y)) = 2 q(y) + 2 q(x).
        f = 2.0 * (np.add.outer(q, np.zeros(n)) + np.add.outer(np.zeros(n), q))
    elif dim == 3:
        u = np.multiply.outer(np.multiply.outer(q, q), q)
        # f[k,j,i] = 2 (q_k q_j + q_k q_i + q_j q_i)
        f = 2.0 * (
            np.einsum("k,j,i->kji", q, q, np.ones(n))
            + np.einsum("k,j,i->kji", q, np.ones(n), q)
            + np.einsum("k,j,i->kji", np.ones(n), q, q)
        )
    else:
        raise ValueError("dim must be 2 or 3")
    return np.ascontiguousarray(u), np.ascontiguousarray(zero_boundary(f))


def uniform_rhs(dim: int, n: int, seed: int) -> np.ndarray:
    """i.i.d. U[-1, 1] right-hand side over all nodes (C order), boundary zeroed.

    Drawn with numpy's PCG64 generator ``default_rng(seed)``.
    """
    check_edge(n)
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, size=(n,) * dim)
    return np.ascontiguousarray(zero_boundary(f))


def random_guess(dim: int, n: int, seed: int) -> np.ndarray:
    """i.i.d. U[-1, 1] initial guess on inner nodes, zero boundary."""
    return uniform_rhs(dim, n, seed)


def _box_mean_axis(g: np.ndarray, axis: int, width: int) -> np.ndarray:
    """Width-`width` centred moving mean along one axis, indices clamped at the edges."""
    half = width // 2
    n = g.shape[axis]
    acc = np.zeros_like(g)
    for off in range(-half, half + 1):
        idx = np.clip(np.arange(n) + off, 0, n - 1)
        acc += np.take(g, idx, axis=axis)
    return acc / float(width)


def varcoef_k(n: int, seed: int, ratio: float = 100.0, width: int = 5, dim: int = 3) -> np.ndarray:
    """Smooth log-normal coefficient field with min k = 1 and max k = ratio.

    g0 ~ N(0, 1) i.i.d. on all nodes, then a separable width-5 box mean along
    each axis (indices clamped at the edges), then k = exp(s (g - min g)) with
    s = ln(ratio) / (max g - min g).
    """
    check_edge(n)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=(n,) * dim)
    for ax in range(dim):
        g = _box_mean_axis(g, ax, width)
    gmin, gmax = float(g.min()), float(g.max())
    s = math.log(ratio) / (gmax - gmin)
    k = np.exp(s * (g - gmin))
    return np.ascontiguousarray(k)


def batch_problem(count: int = 512, seed: int = 3, edges=(65, 129, 257, 513, 1025)):
    """Edges drawn uniformly from `edges`, then one U[-1,1] rhs per grid, same rng in order.

    Returns (list of edges, list of float64 2D arrays with zero boundary).
    """
    rng = np.random.default_rng(seed)
    sizes = [int(e) for e in rng.choice(np.asarray(edges), size=count)]
    rhs = []
    for n in sizes:
        f = rng.uniform(-1.0, 1.0, size=(n, n))
        rhs.append(np.ascontiguousarray(zero_boundary(f)))
    return sizes, rhs


class Request:
    """One synthetic solve request of the serving workload."""

    __slots__ = ("t_arrival", "dim", "n", "seed")

    def __init__(self, t_arrival: float, dim: int, n: int, seed: int):
        self.t_arrival = t_arrival
        self.dim = dim
        self.n = n
        self.seed = seed

    def rhs(self) -> np.ndarray:
        return uniform_rhs(self.dim, self.n, self.seed)

    def __repr__(self) -> str:  # pragma: no cover - debugging aid
        return f"Request(t={self.t_arrival:.6f}, dim={self.dim}, n={self.n}, seed={self.seed})"


def serving_requests(count: int, rate: float, seed: int = 4,
                     edges2d=(257, 513, 1025, 2049), edges3d=(33, 65, 129, 257),
                     frac2d: float = 0.6) -> list[Request]:
    """Poisson arrival stream: exponential inter-arrival times with mean 1/rate.

    Each request is 2D with probability `frac2d` (edge uniform from `edges2d`)
    and 3D otherwise (edge uniform from `edges3d`); its rhs is U[-1, 1] drawn
    from its own seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < frac2d:
            dim, n = 2, int(rng.choice(np.asarray(edges2d)))
        else:
            dim, n = 3, int(rng.choice(np.asarray(edges3d)))
        out.append(Request(t, dim, n, seed * 1_000_003 + r))
    return out


# Cell-centred grids: n = 2**L cells per axis, cell i centred at (i + 1/2) / n,
# C-ordered (n, n) / (n, n, n) arrays, x fastest, no boundary entries.
def cell_centres(n: int) -> np.ndarray:
    """Cell-centre coordinates (i + 1/2) / n."""
    return (np.arange(n, dtype=np.float64) + 0.5) / float(n)


def random_cells(dim: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """U[-scale, scale] on every cell."""
    return np.random.default_rng(seed).uniform(-1, 1, (n,) * dim) * scale


def noisy_image(dim: int, n: int, seed: int, sigma: float = 0.1) -> np.ndarray:
    """The denoising workload of the complex-diffusion form, synthetic: value 1
    inside the disc (2D) or ball (3D) of radius 0.3 about the centre, 0
    outside, plus N(0, sigma^2) noise per cell; complex128 with zero imaginary
    part (the initial state of the diffusion)."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*([cell_centres(n)] * dim), indexing="ij")[::-1]  # x, y[, z]
    r2 = sum((g - 0.5) ** 2 for g in grids)
    img = (r2 < 0.09).astype(np.float64)
    return np.ascontiguousarray((img + sigma * rng.standard_normal(img.shape)).astype(np.complex128))


def random_complex(dim: int, n: int, seed: int, scale: float = 1.0, im: float = 0.3) -> np.ndarray:
    """scale * (U[-1, 1] + i U[-im, im]) on every cell (complex128)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (n,) * dim) + 1j * rng.uniform(-im, im, (n,) * dim)
    return np.ascontiguousarray(a * scale)
