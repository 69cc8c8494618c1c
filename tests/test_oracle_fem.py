"""Pins for the oracle's P1 assembly (paper, Section 2: stiffness and mass
matrices of the P1 state/control space)."""
import math

import numpy as np
import pytest

import inputs
from oracle import fem
from oracle.csr import CSR, transpose

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def dense(a: CSR):
    return a.dense()


def test_2d_stiffness_is_five_point_stencil():
    # kappa = 1 on the diagonal-split square grid: the P1 stiffness is the
    # 5-point Laplacian (4, -1 x 4) and the diagonal couplings are exactly 0
    # but stored (textbook identity for right triangles).
    n = 8
    m = inputs.mesh2d(n)
    A, M = fem.assemble(m.coords, m.elems, inputs.kappa_const(m))
    Ad = dense(A)
    for j in range(1, n):
        for i in range(1, n):
            v = i + (n + 1) * j
            assert Ad[v, v] == 4.0
            for w in (v - 1, v + 1, v - (n + 1), v + (n + 1)):
                assert Ad[v, w] == -1.0
            s, e = A.rowptr[v], A.rowptr[v + 1]
            cols = set(A.col[s:e].tolist())
            # 7-entry row: self, 4 axis neighbours, 2 diagonal neighbours (zero)
            assert cols == {v, v - 1, v + 1, v - (n + 1), v + (n + 1), v + 1 + (n + 1), v - 1 - (n + 1)}
            assert Ad[v, v + n + 2] == 0.0 and Ad[v, v - n - 2] == 0.0


def test_3d_stiffness_is_h_times_seven_point_stencil():
    # Kuhn split of the unit cube with kappa = 1: A = h * (7-point Laplacian).
    n = 4
    h = 1.0 / n
    m = inputs.mesh3d(n)
    A, M = fem.assemble(m.coords, m.elems, inputs.kappa_const(m))
    Ad = dense(A)
    n1 = n + 1
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                v = i + n1 * (j + n1 * k)
                row = Ad[v].copy()
                assert abs(row[v] - 6 * h) < 1e-14
                for s in (1, n1, n1 * n1):
                    assert abs(row[v + s] + h) < 1e-14 and abs(row[v - s] + h) < 1e-14
                    row[v + s] = row[v - s] = 0.0
                row[v] = 0.0
                assert np.max(np.abs(row)) < 1e-14


def test_2d_interior_mass_row():
    n = 8
    h = 1.0 / n
    m = inputs.mesh2d(n)
    _, M = fem.assemble(m.coords, m.elems, inputs.kappa_const(m))
    Md = dense(M)
    v = 3 + (n + 1) * 4
    assert abs(Md[v, v] - h * h / 2) < 1e-16
    nbrs = [v - 1, v + 1, v - (n + 1), v + (n + 1), v + n + 2, v - n - 2]
    for w in nbrs:
        assert abs(Md[v, w] - h * h / 12) < 1e-16
    assert np.count_nonzero(Md[v]) == 7


@pytest.mark.parametrize("mesh", ["2d", "2dj", "3d"])
def test_mass_sums_to_volume_and_stiffness_kills_constants(mesh):
    m = {"2d": lambda: inputs.mesh2d(6), "2dj": lambda: inputs.mesh2d(9, jitter=0.2),
         "3d": lambda: inputs.mesh3d(3)}[mesh]()
    kappa = inputs.kappa_lognormal(m, 1.0) if mesh != "2d" else inputs.kappa_checkerboard(m)
    A, M = fem.assemble(m.coords, m.elems, kappa)
    assert abs(M.val.sum() - 1.0) < 1e-13               # sum_ij M_ij = |Omega|
    ones = np.ones(A.nrows)
    assert np.max(np.abs(A.matvec(ones))) < 1e-12 * np.max(np.abs(A.val))
    t = transpose(A)                                    # exact symmetry
    assert np.array_equal(t.col, A.col) and np.array_equal(t.val, A.val)


def _barycentric_gradients_by_solve(x):
    # independent route: solve [1 x^T] c = e_a for the affine basis functions
    d = x.shape[1]
    V = np.hstack([np.ones((d + 1, 1)), x])
    C = np.linalg.solve(V, np.eye(d + 1))   # column a: coefficients of lambda_a
    return C[1:, :].T                        # (d+1, d)


def _quadrature_mass(x):
    # exact for quadratics: 2D edge-midpoint rule; 3D 4-point degree-2 rule
    d = x.shape[1]
    if d == 2:
        area = abs(np.linalg.det(x[1:] - x[0])) / 2
        pts = [(0.5, 0.5, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5)]
        w = [area / 3] * 3
    else:
        vol = abs(np.linalg.det(x[1:] - x[0])) / 6
        a, b = 0.5854101966249685, 0.1381966011250105
        pts = [(a, b, b, b), (b, a, b, b), (b, b, a, b), (b, b, b, a)]
        w = [vol / 4] * 4
    Me = np.zeros((d + 1, d + 1))
    for lam, wq in zip(pts, w):
        lam = np.array(lam)
        Me += wq * np.outer(lam, lam)
    return Me


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrices_against_independent_formulas(dim):
    m = inputs.mesh2d(5, jitter=0.2) if dim == 2 else inputs.mesh3d(2)
    kappa = np.linspace(0.5, 3.0, m.nelems)
    Ke, Me = fem.element_matrices(m.coords, m.elems, kappa)
    for e in range(0, m.nelems, 3):
        x = m.coords[m.elems[e]]
        g = _barycentric_gradients_by_solve(x)
        vol = abs(np.linalg.det(x[1:] - x[0])) / math.factorial(dim)
        Kref = kappa[e] * vol * g @ g.T
        np.testing.assert_allclose(Ke[e], Kref, rtol=1e-12, atol=1e-14 * np.abs(Kref).max())
        np.testing.assert_allclose(Me[e], _quadrature_mass(x), rtol=1e-12)


def test_dirichlet_stiffness_pattern_counts():
    # nnz of the Dirichlet-reduced stiffness.  On the uniform meshes the diagonal
    # edges carry exactly zero stiffness (right triangles: the edge opposite the
    # right angle; the cubes' tetrahedra likewise), and A_0 keeps no stored
    # zeros: interior rows hold the 5-point (2D) and 7-point (3D) stencils, minus
    # the couplings to Dirichlet nodes, plus one diagonal per Dirichlet node;
    # the mass matrix keeps the full pattern
    m = inputs.mesh2d(32)
    A, M = fem.assemble(m.coords, m.elems, inputs.kappa_const(m))
    A0 = fem.dirichlet_stiffness(A, m.boundary.astype(bool))
    ni = 31
    assert (m.nverts, M.nnz, A0.nnz) == (1089, 7361, ni * ni * 5 - 4 * ni + (1089 - ni * ni))
    m3 = inputs.mesh3d(8)
    A3, M3 = fem.assemble(m3.coords, m3.elems, inputs.kappa_lognormal(m3, 1.0))
    A30 = fem.dirichlet_stiffness(A3, m3.boundary.astype(bool))
    ni = 7
    assert A30.nnz == ni ** 3 * 7 - 6 * ni ** 2 + (m3.nverts - ni ** 3)
    assert A3.nnz == M3.nnz > A30.nnz
    bc = np.nonzero(m.boundary)[0]
    for d in bc[:5]:
        s, e = A0.rowptr[d], A0.rowptr[d + 1]
        assert list(A0.col[s:e]) == [d] and A0.val[s] == 1.0
