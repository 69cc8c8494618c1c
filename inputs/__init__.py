"""Seeded synthetic inputs for the elliptic control problem.

This module only *generates problem data*: meshes (node coordinates, simplex
connectivity, boundary flags), the diffusion coefficient kappa per element,
desired states y_d at the nodes, controls and random directions.  It contains
none of the method's arithmetic (no finite-element integrals, no multigrid, no
Krylov solver), so both the CPU oracle and the GPU library's Python binding may
draw their inputs from it.

Problem statement (paper, Section 2, eqs. functionalcont/pdecont): minimise
1/2||y - y_d||^2 + beta/2 ||u||^2 subject to -div(kappa grad y) = u in the unit
square/cube with y = 0 on the boundary.  The paper's own meshes (a 474-element
tetrahedral mesh refined uniformly, and an engine-bracket mesh) are not
available; structured simplicial meshes of the unit square/cube of the same
node counts stand in for them.

All random draws use numpy.random.default_rng(seed) (PCG64).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

SEED_JITTER = 1
SEED_YD = 2
SEED_KAPPA = 3
SEED_U = 4
SEED_DIR = 5
AGG_SEED = 0x200111533


@dataclass
class Mesh:
    dim: int
    n: int                      # cells per side
    coords: np.ndarray          # (N, dim) float64
    elems: np.ndarray           # (E, dim+1) int32, vertex ids
    boundary: np.ndarray        # (N,) uint8, 1 on the boundary of the unit square/cube

    @property
    def nverts(self) -> int:
        return self.coords.shape[0]

    @property
    def nelems(self) -> int:
        return self.elems.shape[0]


def mesh2d(n: int, jitter: float = 0.0, seed: int = SEED_JITTER) -> Mesh:
    """Uniform n x n grid of the unit square, each cell split into two triangles.

    Node (i, j) sits at (i h, j h), h = 1/n, with id i + (n+1) j.  Cell (i, j)
    (numbered i + n j) holds the triangles {(i,j),(i+1,j),(i+1,j+1)} and
    {(i,j),(i+1,j+1),(i,j+1)}, in that order.  With jitter > 0 every interior
    node coordinate is moved by an independent U[-jitter h, +jitter h] draw,
    drawn node by node, x then y; boundary nodes stay fixed.
    """
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    coords = np.stack([ii * h, jj * h], axis=1).astype(np.float64)
    boundary = ((ii == 0) | (ii == n) | (jj == 0) | (jj == n)).astype(np.uint8)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        interior = np.nonzero(boundary == 0)[0]
        d = rng.uniform(-jitter * h, jitter * h, size=(interior.size, 2))
        coords[interior] += d
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = ci + (n + 1) * cj
    v10 = v00 + 1
    v11 = v00 + 1 + (n + 1)
    v01 = v00 + (n + 1)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    elems = np.empty((2 * n * n, 3), dtype=np.int32)
    elems[0::2] = t1
    elems[1::2] = t2
    m = Mesh(2, n, coords, elems, boundary)
    if jitter > 0.0:
        x = coords[elems]
        det = ((x[:, 1, 0] - x[:, 0, 0]) * (x[:, 2, 1] - x[:, 0, 1])
               - (x[:, 1, 1] - x[:, 0, 1]) * (x[:, 2, 0] - x[:, 0, 0]))
        assert np.all(det > 0.0), "jittered mesh has an inverted triangle"
    return m


KUHN_PERMS = list(itertools.permutations(range(3)))  # lexicographic order


def mesh3d(n: int) -> Mesh:
    """Uniform n^3 grid of the unit cube, each cube split into 6 Kuhn tetrahedra.

    Node (i, j, k) has id i + (n+1)(j + (n+1) k).  Cube c (numbered
    i + n (j + n k)) with lower corner v0 yields, for each permutation pi of
    (x, y, z) in lexicographic order, the tetrahedron v0, v1 = v0 + e_pi1,
    v2 = v1 + e_pi2, v3 = v0 + (1,1,1).  The split is conforming.
    """
    h = 1.0 / n
    n1 = n + 1
    kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    kk = kk.ravel()
    coords = np.stack([ii * h, jj * h, kk * h], axis=1).astype(np.float64)
    boundary = ((ii == 0) | (ii == n) | (jj == 0) | (jj == n) | (kk == 0) | (kk == n)).astype(np.uint8)
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (ci + n1 * (cj + n1 * ck)).ravel().astype(np.int64)
    step = np.array([1, n1, n1 * n1], dtype=np.int64)
    elems = np.empty((6 * base.size, 4), dtype=np.int32)
    for p, perm in enumerate(KUHN_PERMS):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v0 + step.sum()
        elems[p::6] = np.stack([v0, v1, v2, v3], axis=1)
    return Mesh(3, n, coords, elems, boundary)


def centroids(mesh: Mesh) -> np.ndarray:
    return mesh.coords[mesh.elems].mean(axis=1)


def kappa_const(mesh: Mesh, value: float = 1.0) -> np.ndarray:
    return np.full(mesh.nelems, value, dtype=np.float64)


def kappa_checkerboard(mesh: Mesh, lo: float = 1.0, hi: float = 1e3, cells: int = 4) -> np.ndarray:
    """Piecewise-constant kappa on a cells x cells checkerboard, evaluated at the
    element centroid: square (p, q) = (floor(4 x_c), floor(4 y_c)) gets lo when
    p + q is even and hi when it is odd."""
    c = centroids(mesh)
    p = np.minimum(np.floor(cells * c[:, 0]).astype(np.int64), cells - 1)
    q = np.minimum(np.floor(cells * c[:, 1]).astype(np.int64), cells - 1)
    return np.where((p + q) % 2 == 0, lo, hi).astype(np.float64)


def kappa_lognormal(mesh: Mesh, sigma2: float, seed: int = SEED_KAPPA, modes: int = 16,
                    kmax: int = 4) -> np.ndarray:
    """kappa = exp(g), g = sqrt(2 sigma2 / modes) sum_m cos(2 pi w_m . x + phi_m),
    at the element centroid.  w_m is uniform over the nonzero integer vectors of
    [-kmax, kmax]^d and phi_m ~ U[0, 2 pi); the pointwise variance of g is sigma2."""
    d = mesh.dim
    rng = np.random.default_rng(seed)
    grid = np.array(list(itertools.product(range(-kmax, kmax + 1), repeat=d)), dtype=np.float64)
    grid = grid[np.any(grid != 0, axis=1)]
    idx = rng.integers(0, grid.shape[0], size=modes)
    w = grid[idx]
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    c = centroids(mesh)
    g = np.zeros(c.shape[0])
    for m in range(modes):
        g += np.cos(2.0 * math.pi * (c @ w[m]) + phi[m])
    g *= math.sqrt(2.0 * sigma2 / modes)
    return np.exp(g)


def kappa_ball(mesh: Mesh, alpha: float, radius: float = 0.25) -> np.ndarray:
    """kappa = alpha inside the ball |x - centre| <= radius, 1 outside (centroid rule)."""
    c = centroids(mesh)
    r = np.linalg.norm(c - 0.5, axis=1)
    return np.where(r <= radius, alpha, 1.0).astype(np.float64)


def yd_sin(mesh: Mesh, scale: float = 1.0) -> np.ndarray:
    """Nodal interpolant of scale * prod_i sin(pi x_i)."""
    v = np.ones(mesh.nverts)
    for a in range(mesh.dim):
        v = v * np.sin(math.pi * mesh.coords[:, a])
    return scale * v


def yd_manufactured(mesh: Mesh, beta: float) -> np.ndarray:
    """Desired state with a closed-form optimal control (paper, eq. test-state):
    y_d = (1/(d pi^2) + d pi^2 beta) prod sin(pi x_i), whose optimal control is
    u* = prod sin(pi x_i) for the continuous problem with kappa = 1."""
    d = mesh.dim
    return yd_sin(mesh, 1.0 / (d * math.pi ** 2) + d * math.pi ** 2 * beta)


def yd_bumps(mesh: Mesh, seed: int = SEED_YD, count: int = 8, width: float = 0.05) -> np.ndarray:
    """sum_m a_m exp(-|x - c_m|^2 / (2 width^2)), a_m ~ U[0,1], c_m ~ U[0,1]^d."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=count)
    c = rng.uniform(0.0, 1.0, size=(count, mesh.dim))
    v = np.zeros(mesh.nverts)
    for m in range(count):
        r2 = np.sum((mesh.coords - c[m]) ** 2, axis=1)
        v += a[m] * np.exp(-r2 / (2.0 * width * width))
    return v


def controls(nverts: int, nb: int, seed: int = SEED_U) -> np.ndarray:
    """u ~ N(0, 1) at every node, nb columns, row-major (N, nb)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nverts, nb))


def directions(nverts: int, count: int, seed: int = SEED_DIR) -> np.ndarray:
    """count unit-2-norm directions, rows of shape (count, N)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, nverts))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@dataclass
class Problem:
    name: str
    mesh: Mesh
    kappa: np.ndarray
    beta: float
    yd: np.ndarray              # (N, nb)
    dirichlet: np.ndarray       # (N,) uint8
    extra: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return self.yd.shape[1]


def _col(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 1))


def ball_problem(n: int, alpha: float) -> Problem:
    """The varying-coefficient setting of the paper's Section 5.6 on the n^3
    Kuhn cube: kappa = alpha inside the ball of radius 1/4 about the centre and
    1 outside, Dirichlet nodes only on the face z = 0 (homogeneous Neumann on
    the others), y_d = 1, beta = 1."""
    m = mesh3d(n)
    face = (m.coords[:, 2] == 0.0).astype(np.uint8)
    return Problem(f"ball{alpha:g}", m, kappa_ball(m, alpha), 1.0, np.ones((m.nverts, 1)), face)


def config(name: str, n: int | None = None, nb: int | None = None) -> Problem:
    """The five workloads, optionally at a reduced grid size n (for tests).

    c1  2D 32x32, kappa = 1, beta = 1e-2, y_d = sin(pi x) sin(pi y)
    c2  2D 256x256 jittered (+-0.2h), 4x4 checkerboard kappa in {1, 1e3},
        beta = 1e-2 (c2b: 1e-4), y_d = 8 seeded Gaussian bumps
    c3  3D 64^3 Kuhn tets, log-normal kappa (variance 1), beta = 1e-3,
        y_d = the manufactured state of eq. test-state
    c4  c2 mesh and kappa, beta = 1e-2, y_d = bumps; 8 controls N(0,1) and 20
        unit directions for the gradient check
    c5  3D 128^3, log-normal kappa (variance 2), beta = 1e-4, 16 bump y_d
        (seeds 2..17)
    """
    if name == "c1":
        m = mesh2d(n or 32)
        return Problem(name, m, kappa_const(m), 1e-2, _col(yd_sin(m)), m.boundary)
    if name in ("c2", "c2b"):
        m = mesh2d(n or 256, jitter=0.2)
        beta = 1e-2 if name == "c2" else 1e-4
        return Problem(name, m, kappa_checkerboard(m), beta, _col(yd_bumps(m)), m.boundary)
    if name == "c3":
        m = mesh3d(n or 64)
        beta = 1e-3
        yd = _col(yd_manufactured(m, beta))
        if nb:
            yd = np.concatenate([yd] + [_col(yd_bumps(m, SEED_YD + k)) for k in range(nb - 1)], axis=1)
        return Problem(name, m, kappa_lognormal(m, 1.0), beta, yd, m.boundary)
    if name == "c4":
        m = mesh2d(n or 256, jitter=0.2)
        p = Problem(name, m, kappa_checkerboard(m), 1e-2, _col(yd_bumps(m)), m.boundary)
        p.extra["u"] = controls(m.nverts, 8)
        p.extra["dirs"] = directions(m.nverts, 20)
        p.extra["fd_step"] = 1e-6
        return p
    if name == "c5":
        m = mesh3d(n or 128)
        k = nb or 16
        yd = np.stack([yd_bumps(m, SEED_YD + i) for i in range(k)], axis=1)
        return Problem(name, m, kappa_lognormal(m, 2.0), 1e-4, np.ascontiguousarray(yd), m.boundary)
    raise ValueError(f"unknown config {name!r}")
