"""P1 finite-element assembly (oracle; test infrastructure only).

Paper, Section 2: the stiffness matrix [A]_ij = a(phi_j, phi_i) with
a(y, v) = int kappa grad y . grad v, and the mass matrices [M]_ij =
(phi_j, phi_i).  State and control use the same P1 space; only the boundary
condition differs (the state lives in H^1_0).

Element formulas (textbook P1 on a d-simplex T with vertices x_0..x_d):
  * J has rows x_a - x_0 (a = 1..d); the gradient of the barycentric
    coordinate lambda_a (a >= 1) is column a of J^{-1}, and
    grad lambda_0 = -(sum of the others);
  * K_T[a, b] = kappa_T |T| grad lambda_a . grad lambda_b;
  * M_T[a, b] = |T| (1 + delta_ab) / ((d+1)(d+2)).
J^{-1} is formed from the adjugate divided by det J.  Every global entry sums
its element contributions in ascending element index, left to right.  The
sparsity pattern is the mesh graph (all vertex pairs sharing an element),
sorted, with explicit zeros kept.
"""
from __future__ import annotations

import numpy as np

from .csr import CSR, sum_by_key


def element_gradients(coords: np.ndarray, elems: np.ndarray):
    """Return (grads (E, d+1, d), measure (E,)) for every simplex."""
    X = coords[elems]                      # (E, d+1, d)
    d = coords.shape[1]
    J = X[:, 1:, :] - X[:, 0:1, :]         # rows: edge vectors x_a - x_0
    if d == 2:
        j00, j01 = J[:, 0, 0], J[:, 0, 1]
        j10, j11 = J[:, 1, 0], J[:, 1, 1]
        det = j00 * j11 - j01 * j10
        inv = np.empty_like(J)
        inv[:, 0, 0] = j11 / det
        inv[:, 0, 1] = -j01 / det
        inv[:, 1, 0] = -j10 / det
        inv[:, 1, 1] = j00 / det
        meas = np.abs(det) / 2.0
    elif d == 3:
        a, b, c = J[:, 0, 0], J[:, 0, 1], J[:, 0, 2]
        e, f, g = J[:, 1, 0], J[:, 1, 1], J[:, 1, 2]
        h, i, k = J[:, 2, 0], J[:, 2, 1], J[:, 2, 2]
        c00 = f * k - g * i
        c01 = g * h - e * k
        c02 = e * i - f * h
        det = a * c00 + b * c01 + c * c02
        inv = np.empty_like(J)
        # inverse = adjugate / det; adjugate[r, s] = cofactor[s, r]
        inv[:, 0, 0] = c00 / det
        inv[:, 0, 1] = (c * i - b * k) / det
        inv[:, 0, 2] = (b * g - c * f) / det
        inv[:, 1, 0] = c01 / det
        inv[:, 1, 1] = (a * k - c * h) / det
        inv[:, 1, 2] = (c * e - a * g) / det
        inv[:, 2, 0] = c02 / det
        inv[:, 2, 1] = (b * h - a * i) / det
        inv[:, 2, 2] = (a * f - b * e) / det
        meas = np.abs(det) / 6.0
    else:
        raise ValueError("dimension must be 2 or 3")
    grads = np.empty((elems.shape[0], d + 1, d))
    for a_ in range(1, d + 1):
        grads[:, a_, :] = inv[:, :, a_ - 1]
    g0 = -grads[:, 1, :]
    for a_ in range(2, d + 1):
        g0 = g0 - grads[:, a_, :]
    grads[:, 0, :] = g0
    return grads, meas


def element_matrices(coords: np.ndarray, elems: np.ndarray, kappa: np.ndarray):
    """Element stiffness (E, d+1, d+1) and mass (E, d+1, d+1)."""
    d = coords.shape[1]
    grads, meas = element_gradients(coords, elems)
    w = kappa * meas
    nl = d + 1
    Ke = np.empty((elems.shape[0], nl, nl))
    for p in range(nl):
        for q in range(nl):
            dot = grads[:, p, 0] * grads[:, q, 0]
            for c in range(1, d):
                dot = dot + grads[:, p, c] * grads[:, q, c]
            Ke[:, p, q] = w * dot
    base = meas / float((d + 1) * (d + 2))
    Me = np.empty_like(Ke)
    for p in range(nl):
        for q in range(nl):
            Me[:, p, q] = 2.0 * base if p == q else base
    return Ke, Me


def assemble(coords: np.ndarray, elems: np.ndarray, kappa: np.ndarray):
    """Global stiffness A and mass M (no boundary conditions), as CSR."""
    n = coords.shape[0]
    Ke, Me = element_matrices(coords, elems, kappa)
    nl = elems.shape[1]
    rows = np.repeat(elems.astype(np.int64), nl, axis=1).ravel()    # (e, a, b) -> elems[e, a]
    cols = np.tile(elems.astype(np.int64), (1, nl)).ravel()         # (e, a, b) -> elems[e, b]
    A = sum_by_key(rows, cols, Ke.ravel(), n, n)
    M = sum_by_key(rows, cols, Me.ravel(), n, n)
    return A, M


def dirichlet_stiffness(A: CSR, dirichlet: np.ndarray) -> CSR:
    """A_0 = D A D + (I - D), D = diag(1 - dirichlet): Dirichlet rows and
    columns are removed from the pattern and the Dirichlet diagonal is 1.
    This is the state space Y in H^1_0 of Section 2 written on all nodes.
    Stored zeros of A are not entries of A_0: an off-diagonal entry is kept
    only when it is nonzero (on the uniform meshes the diagonal edges of the
    triangles and of the cubes' tetrahedra carry exactly zero stiffness)."""
    bc = dirichlet.astype(bool)
    r = A.rows()
    keep = ~bc[r] & ~bc[A.col] & ((A.val != 0.0) | (r == A.col))
    rr = np.concatenate([r[keep], np.nonzero(bc)[0]])
    cc = np.concatenate([A.col[keep], np.nonzero(bc)[0]])
    vv = np.concatenate([A.val[keep], np.ones(int(bc.sum()))])
    order = np.lexsort((cc, rr))
    rr, cc, vv = rr[order], cc[order], vv[order]
    rowptr = np.zeros(A.nrows + 1, dtype=np.int64)
    np.add.at(rowptr, rr + 1, 1)
    return CSR(np.cumsum(rowptr), cc, vv, A.ncols)
