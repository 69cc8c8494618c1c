"""Explicit dense operators for tiny meshes (oracle; test infrastructure only).

These follow the paper's own formulation in the M_u inner product, before the
practical rewrite of Section 5.2, so that the sparse recursive code in
oracle.solve can be checked against an independent statement:

  K_j   = A_j^{-1} M_{yu,j}                       (eq. solutionopdef)
  K_j^* = M_{u,j}^{-1} K_j^T M_{y,j}              (Section 2)
  G_j   = K_j^* K_j + beta I                      (eq. truefirstorder)
  Pi_j  = M_{u,j+1}^{-1} P_j^T M_{u,j}            (L2 projection, Section 3.1)
  T_j^{-1} = P_j W_{j+1} Pi_j + beta^{-1}(I - P_j Pi_j)   (eq. twogridinmulti)
  W_{l-1} = G_{l-1}^{-1};  W_j = 2 T_j^{-1} - T_j^{-1} G_j T_j^{-1} (0<j<l-1);
  W_0 = T_0^{-1}           (eqs. twogridinmultiactual, ...fine)

with P_j = S_j (the prolongators of oracle.sa).  The practical-form
preconditioner of the sparse code is B_0 = W_0 M_{u,0}^{-1}.
"""
from __future__ import annotations

import numpy as np

from . import sa


def level_ops(h: sa.Hierarchy, j: int):
    A, My, Mu, Myu = sa.dense_level_matrices(h, j)
    K = np.linalg.solve(A, Myu)
    Kstar = np.linalg.solve(Mu, K.T @ My)
    G = Kstar @ K + h.opts.beta * np.eye(A.shape[0])
    return dict(A=A, My=My, Mu=Mu, Myu=Myu, K=K, Kstar=Kstar, G=G)


def projection(h: sa.Hierarchy, j: int) -> np.ndarray:
    P = h.levels[j].S.dense()
    Mu = level_ops(h, j)["Mu"]
    Mu1 = level_ops(h, j + 1)["Mu"]
    return np.linalg.solve(Mu1, P.T @ Mu)


def W(h: sa.Hierarchy, j: int, ell: int) -> np.ndarray:
    """The multilevel approximation W_j of G_j^{-1} (paper, Section 3.2)."""
    ops = level_ops(h, j)
    if j == ell - 1:
        return np.linalg.inv(ops["G"])
    P = h.levels[j].S.dense()
    Pi = projection(h, j)
    n = P.shape[0]
    Tinv = P @ W(h, j + 1, ell) @ Pi + (1.0 / h.opts.beta) * (np.eye(n) - P @ Pi)
    if j == 0:
        return Tinv
    return 2.0 * Tinv - Tinv @ ops["G"] @ Tinv


def two_grid_T(h: sa.Hierarchy, j: int):
    """T_j = P G_{j+1} Pi + beta (I - P Pi) and its stated inverse (eqs.
    twogriddirect and twogrid)."""
    P = h.levels[j].S.dense()
    Pi = projection(h, j)
    G1 = level_ops(h, j + 1)["G"]
    n = P.shape[0]
    beta = h.opts.beta
    T = P @ G1 @ Pi + beta * (np.eye(n) - P @ Pi)
    Tinv = P @ np.linalg.inv(G1) @ Pi + (1.0 / beta) * (np.eye(n) - P @ Pi)
    return T, Tinv


def hessian_practical(h: sa.Hierarchy, j: int = 0) -> np.ndarray:
    """H_j = M_{u,j} G_j = K^T M_y K + beta M_u (eq. firstorderpractice)."""
    ops = level_ops(h, j)
    return ops["K"].T @ ops["My"] @ ops["K"] + h.opts.beta * ops["Mu"]


def rhs_practical(h: sa.Hierarchy, yd: np.ndarray) -> np.ndarray:
    ops = level_ops(h, 0)
    return ops["K"].T @ ops["My"] @ yd


def vcycle_matrix(apply, n: int) -> np.ndarray:
    """Columns of an operator applied to the unit vectors."""
    return np.stack([apply(e) for e in np.eye(n)], axis=1)


def quality(h: sa.Hierarchy, j: int):
    """(a_j, a~_j): a_j = ||M_y^{1/2} E M_u^{-1/2}||_2 (eq. ajnumerical, with
    symmetric square roots of the level's mass matrices) and a~_j = ||E||_2
    (eq. aj-tilde), E = K_j - S_j K_{j+1} Pi_j, both by singular values."""
    o0, o1 = level_ops(h, j), level_ops(h, j + 1)
    E = o0["K"] - h.levels[j].S.dense() @ o1["K"] @ projection(h, j)

    def sqrt_spd(B):
        w, V = np.linalg.eigh(0.5 * (B + B.T))
        return (V * np.sqrt(np.clip(w, 0.0, None))) @ V.T

    My_half = sqrt_spd(o0["My"])
    Mu_half = sqrt_spd(o0["Mu"])
    a = np.linalg.norm(My_half @ E @ np.linalg.inv(Mu_half), 2)
    return float(a), float(np.linalg.norm(E, 2))
