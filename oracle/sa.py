"""Smoothed-aggregation AMG hierarchy (oracle; test infrastructure only).

The paper fixes ideas on smoothed aggregation (Section 3.1, citing Vanek,
Mandel and Brezina) and only needs from the AMG: prolongators S_j (state) and
P_j (control) and the Galerkin matrices of eqs. coarsestiffness/coarsemass,
A_{j+1} = S_j^T A_j S_j, M_{y,j+1} = S_j^T M_{y,j} S_j, M_{u,j+1} = P_j^T
M_{u,j} P_j, M_{yu,j+1} = S_j^T M_{yu,j} P_j.  The paper's own BoomerAMG
parameters are not given, so the aggregation is specified here to the level of
operation order (readings recorded with the design notes):

  strength   k != i strong iff neither node is Dirichlet and
             a_ik*a_ik >= t*(a_ii*a_kk), t = theta_j*theta_j,
             theta_j = 0.08 * 0.5**j  (three roundings, no fused multiply-add)
  roots      greedy distance-2 maximal independent set of the strong graph,
             visiting nodes by decreasing key (splitmix64(seed ^ (j<<40) ^ i), i)
  numbering  coarse id of a root = number of roots with a smaller node index
  phase 2    a non-root with a strong root neighbour joins the root r with the
             largest |a_ir| (ties: smallest r)
  phase 3    every other non-Dirichlet node joins agg(k) of its strong
             neighbour k assigned in phase 2 with the largest |a_ik| (ties:
             smallest k)
  smoothing  S = (I - omega D^{-1} A) P_tent, P_tent[i, agg(i)] = 1,
             omega = (4/3)/rho, rho = max_i (sum_k |a_ik|)/a_ii;
             S[i,J] = [agg(i)=J] - (omega*s_iJ)/a_ii with
             s_iJ = sum over k ascending with agg(k)=J of a_ik
  Galerkin   T = A S summed over k ascending, then S^T T over i ascending
             (S^T stored explicitly by a stable transpose); the lower triangle
             is then copied from the upper one so every coarse matrix is
             exactly symmetric
  control    P_j = S_j, so with the Dirichlet reading of Section 2
             (M_y = DMD, M_yu = DM, M_u = M at level 0) all four coarse mass
             matrices coincide: M_{j+1} = S_j^T M_j S_j
  stop       level j is the coarsest when n_j <= max_coarse, when
             j + 1 = max_levels, or when n_{j+1} > 0.9 n_j
  small      on coarse levels (j >= 1) with n_j <= dense_solve_max the
             A_j- and M_j-solves are exact (dense Cholesky) instead of
             iterative; they return what the iterative solves approximate.
             This includes the M-solves of the coarsest level (whose A-solves
             are always dense).  A V-cycle that reaches such a level solves
             there exactly and goes no deeper (the levels below serve the
             Hessian levels only)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .csr import CSR, ordered_segment_sum, sum_by_key, transpose

U64 = np.uint64
_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014) applied
    to each 64-bit word: add the golden gamma, then two xor-shift-multiply
    rounds and a final xor-shift."""
    with np.errstate(over="ignore"):
        z = x.astype(U64) + U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> U64(30))) * U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> U64(27))) * U64(0x94D049BB133111EB)
        z = z ^ (z >> U64(31))
    return z


def priority_hash(n: int, level: int, seed: int) -> np.ndarray:
    base = U64((seed ^ (level << 40)) & _M64)
    return splitmix64(base ^ np.arange(n, dtype=U64))


def strength(A: CSR, theta: float, dirichlet: np.ndarray) -> np.ndarray:
    """Boolean flag per stored entry of A: is (i, k) a strong connection."""
    r = A.rows()
    d = A.diag()
    t = theta * theta
    aik = A.val
    lhs = aik * aik
    rhs = t * (d[r] * d[A.col])
    return (r != A.col) & ~dirichlet[r] & ~dirichlet[A.col] & (lhs >= rhs)


def strong_graph(A: CSR, flags: np.ndarray) -> CSR:
    r = A.rows()
    rr = r[flags]
    cc = A.col[flags]
    rowptr = np.zeros(A.nrows + 1, dtype=np.int64)
    np.add.at(rowptr, rr + 1, 1)
    return CSR(np.cumsum(rowptr), cc, A.val[flags], A.ncols)


def mis2_greedy(G: CSR, keys: np.ndarray, active: np.ndarray) -> np.ndarray:
    """Greedy distance-2 independent set: visit active nodes by decreasing
    (key, index); a node becomes a root iff no root lies within two hops of
    the graph G.  Returns a boolean root flag per node."""
    n = G.nrows
    idx = np.nonzero(active)[0]
    # decreasing (key, i): sort ascending on (i, key) lexicographic then reverse
    order = idx[np.lexsort((idx, keys[idx]))][::-1]
    blocked = np.zeros(n, dtype=bool)
    root = np.zeros(n, dtype=bool)
    rp, cl = G.rowptr, G.col
    for i in order:
        if blocked[i]:
            continue
        root[i] = True
        blocked[i] = True
        nb1 = cl[rp[i]:rp[i + 1]]
        blocked[nb1] = True
        for k in nb1:
            blocked[cl[rp[k]:rp[k + 1]]] = True
    return root


def mis2_rounds(G: CSR, keys: np.ndarray, active: np.ndarray) -> np.ndarray:
    """The same set computed by fixed-priority rounds: an undecided node is
    taken when its (key, index) is the largest among undecided nodes within two
    hops; nodes within two hops of a taken node are then excluded.  Used only to
    pin the equivalence with mis2_greedy in the tests."""
    n = G.nrows
    r = G.rows()
    UNDEC, ROOT, OUT = 0, 1, 2
    state = np.where(active, UNDEC, OUT)
    rank = np.empty(n, dtype=np.int64)          # position in ascending (key, index)
    ordr = np.lexsort((np.arange(n), keys))
    rank[ordr] = np.arange(n)
    while np.any(state == UNDEC):
        val = np.where(state == UNDEC, rank, -1)
        m1 = val.copy()
        np.maximum.at(m1, r, val[G.col])
        m2 = m1.copy()
        np.maximum.at(m2, r, m1[G.col])
        new = (state == UNDEC) & (m2 == rank)
        state[new] = ROOT
        isr = (state == ROOT).astype(np.int8)
        h1 = isr.copy()
        np.maximum.at(h1, r, isr[G.col])
        h2 = h1.copy()
        np.maximum.at(h2, r, h1[G.col])
        state[(state == UNDEC) & (h2 > 0)] = OUT
    return state == ROOT


def aggregate(A: CSR, G: CSR, root: np.ndarray, dirichlet: np.ndarray):
    """Phases 2 and 3 and coarse numbering.  Returns (agg, nc) with agg = -1 on
    Dirichlet nodes."""
    n = A.nrows
    cid = np.cumsum(root) - 1
    agg = np.full(n, -1, dtype=np.int64)
    agg[root] = cid[root]
    gr = G.rows()
    absv = np.abs(G.val)
    # phase 2
    cand = root[G.col] & ~root[gr]
    ci, ck, ca = gr[cand], G.col[cand], absv[cand]
    o = np.lexsort((ck, -ca, ci))
    ci, ck = ci[o], ck[o]
    first = np.ones(ci.size, dtype=bool)
    first[1:] = ci[1:] != ci[:-1]
    p2 = np.zeros(n, dtype=bool)
    agg[ci[first]] = agg[ck[first]]
    p2[ci[first]] = True
    # phase 3
    left = (agg < 0) & ~dirichlet
    cand = left[gr] & p2[G.col]
    ci, ck, ca = gr[cand], G.col[cand], absv[cand]
    o = np.lexsort((ck, -ca, ci))
    ci, ck = ci[o], ck[o]
    first = np.ones(ci.size, dtype=bool)
    first[1:] = ci[1:] != ci[:-1]
    agg[ci[first]] = agg[ck[first]]
    if np.any((agg < 0) & ~dirichlet):
        raise RuntimeError("aggregation left a node unassigned")
    return agg, int(root.sum())


def l1_diag(A: CSR) -> np.ndarray:
    """sum_k |a_ik| in ascending column order (the l1-Jacobi diagonal)."""
    return ordered_segment_sum(np.abs(A.val), A.rowptr)


def smooth_prolongator(A: CSR, agg: np.ndarray, nc: int, dirichlet: np.ndarray):
    """S = (I - omega D^{-1} A) P_tent with the ordered sums of the module doc.
    Returns (S, omega, rho)."""
    d = A.diag()
    rs = l1_diag(A)
    nd = ~dirichlet
    rho = float(np.max(rs[nd] / d[nd])) if nd.any() else 1.0
    omega = (4.0 / 3.0) / rho
    r = A.rows()
    J = agg[A.col]
    keep = nd[r] & (J >= 0)
    S0 = sum_by_key(r[keep], J[keep], A.val[keep], A.nrows, nc)   # s_iJ, ordered over k
    sr = S0.rows()
    v = (omega * S0.val) / d[sr]
    delta = np.where(agg[sr] == S0.col, 1.0, 0.0)
    S = CSR(S0.rowptr, S0.col, delta - v, nc)
    return S, omega, rho


def spgemm_ordered(A: CSR, B: CSR) -> CSR:
    """C = A B, each C[i, J] summed over the stored A[i, k] in ascending k of the
    rounded products A[i, k] * B[k, J] (only stored B[k, J] contribute)."""
    r = A.rows()
    k = A.col
    cnt = B.rowptr[k + 1] - B.rowptr[k]
    total = int(cnt.sum())
    rep_i = np.repeat(r, cnt)
    rep_a = np.repeat(A.val, cnt)
    start = np.repeat(B.rowptr[k], cnt)
    offs = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    bidx = start + offs
    return sum_by_key(rep_i, B.col[bidx], rep_a * B.val[bidx], A.nrows, B.ncols)


def mirror_upper(C: CSR) -> CSR:
    """Copy every strictly-upper value onto its lower-triangle mirror (the
    pattern is symmetric)."""
    t = transpose(C)
    assert np.array_equal(t.rowptr, C.rowptr) and np.array_equal(t.col, C.col)
    r = C.rows()
    val = np.where(r > C.col, t.val, C.val)
    return CSR(C.rowptr, C.col, val, C.ncols)


def galerkin(S: CSR, St: CSR, A: CSR) -> CSR:
    T = spgemm_ordered(A, S)
    C = spgemm_ordered(St, T)
    return mirror_upper(C)


@dataclass
class Opts:
    beta: float = 1e-2
    hess_levels: int = 0            # 0: all AMG levels
    auto_levels: int = 1
    max_levels: int = 10
    max_coarse: int = 200
    dense_max: int = 4096
    dense_solve_max: int = 2048     # coarse levels j >= 1 this small: exact dense A_j and M_j solves
    theta0: float = 0.08
    agg_seed: int = 0x200111533
    nu: int = 1
    smoother: int = 0               # 0 = l1-Jacobi, 1 = Chebyshev of degree 2 (pre and post)
    inner_rtol: float = 1e-8        # the A-solves that apply K and K* (Section 5.3)
    mass_rtol: float = 1e-8          # the paper's mass-solve tolerance (Section 5.3)
    precond_inner_rtol: float = 1e-8 # A-solves inside the preconditioner's H_j, as the paper's inner solves
    inner_maxit: int = 500
    mass_maxit: int = 500
    outer_maxit: int = 200
    coarse_hess_rtol: float = 1e-4
    inner32_rtol: float = 1e-6
    refine_maxit: int = 6
    mixed_mode: int = 0             # float32 path: 0 = FP64 CG with the float32 V-cycle, 1 = refinement
    precond: int = 1                # 0: unpreconditioned outer CG


@dataclass
class Level:
    A: CSR
    M: CSR
    dirichlet: np.ndarray
    dl1: np.ndarray
    S: CSR | None = None
    St: CSR | None = None
    agg: np.ndarray | None = None
    root: np.ndarray | None = None
    strong: np.ndarray | None = None
    omega: float = 0.0
    rho: float = 0.0
    chol_A: tuple | None = None     # dense factors on small coarse levels
    chol_M: tuple | None = None

    @property
    def n(self) -> int:
        return self.A.nrows


@dataclass
class Hierarchy:
    levels: list
    opts: Opts
    chol_A: tuple | None = None          # dense Cholesky of the coarsest A
    ell: int = 0                          # Hessian levels used by the preconditioner
    H_dense: np.ndarray | None = None     # practical-form Hessian at level ell-1
    chol_H: tuple | None = None
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return len(self.levels)


def build(A0: CSR, M: CSR, dirichlet: np.ndarray, opts: Opts) -> Hierarchy:
    """Build the SA hierarchy from the Dirichlet-reduced stiffness A0 (see
    fem.dirichlet_stiffness) and the unmasked mass matrix M."""
    bc = dirichlet.astype(bool)
    levels = [Level(A0, M, bc, l1_diag(A0))]
    j = 0
    while True:
        lev = levels[-1]
        if lev.n <= opts.max_coarse or j + 1 >= opts.max_levels:
            break
        theta = opts.theta0 * 0.5 ** j
        flags = strength(lev.A, theta, lev.dirichlet)
        G = strong_graph(lev.A, flags)
        keys = priority_hash(lev.n, j, opts.agg_seed)
        root = mis2_greedy(G, keys, ~lev.dirichlet)
        agg, nc = aggregate(lev.A, G, root, lev.dirichlet)
        if nc == 0 or nc > 0.9 * lev.n:
            break
        S, omega, rho = smooth_prolongator(lev.A, agg, nc, lev.dirichlet)
        St = transpose(S)
        Ac = galerkin(S, St, lev.A)
        Mc = galerkin(S, St, lev.M)
        lev.S, lev.St, lev.agg, lev.root, lev.strong = S, St, agg, root, flags
        lev.omega, lev.rho = omega, rho
        levels.append(Level(Ac, Mc, np.zeros(nc, dtype=bool), l1_diag(Ac)))
        j += 1
    h = Hierarchy(levels, opts)
    for j in range(1, len(levels) - 1):
        lev = levels[j]
        if lev.n <= opts.dense_solve_max:
            lev.chol_A = sla.cho_factor(lev.A.dense(), lower=True)
            lev.chol_M = sla.cho_factor(lev.M.dense(), lower=True)
    last = levels[-1]
    if last.n > opts.dense_max:
        raise RuntimeError("coarsest level too large for the dense factor")
    h.chol_A = sla.cho_factor(last.A.dense(), lower=True)
    if len(levels) > 1 and last.n <= opts.dense_solve_max:
        last.chol_M = sla.cho_factor(last.M.dense(), lower=True)
    set_hessian_levels(h, opts.hess_levels or h.L)
    return h


# ---- level operators (Section 2 with the Dirichlet reading: M_y = DMD,
# M_yu = DM, M_u = M at level 0; one mass matrix on coarse levels) ----

def mass_u(h: Hierarchy, j: int, x):
    return h.levels[j].M.matvec(x)


def mass_y(h: Hierarchy, j: int, x):
    lev = h.levels[j]
    if j == 0 and lev.dirichlet.any():
        keep = (~lev.dirichlet).astype(np.float64)
        keep = keep.reshape((-1,) + (1,) * (np.ndim(x) - 1))
        return keep * lev.M.matvec(keep * x)
    return lev.M.matvec(x)


def mass_yu(h: Hierarchy, j: int, x):
    lev = h.levels[j]
    if j == 0 and lev.dirichlet.any():
        keep = (~lev.dirichlet).astype(np.float64).reshape((-1,) + (1,) * (np.ndim(x) - 1))
        return keep * lev.M.matvec(x)
    return lev.M.matvec(x)


def mass_yu_t(h: Hierarchy, j: int, x):
    lev = h.levels[j]
    if j == 0 and lev.dirichlet.any():
        keep = (~lev.dirichlet).astype(np.float64).reshape((-1,) + (1,) * (np.ndim(x) - 1))
        return lev.M.matvec(keep * x)
    return lev.M.matvec(x)


def dense_level_matrices(h: Hierarchy, j: int):
    """Dense A_j, M_{y,j}, M_{u,j}, M_{yu,j}."""
    lev = h.levels[j]
    A = lev.A.dense()
    M = lev.M.dense()
    if j == 0 and lev.dirichlet.any():
        D = np.diag((~lev.dirichlet).astype(np.float64))
        return A, D @ M @ D, M, D @ M
    return A, M, M, M


def set_hessian_levels(h: Hierarchy, ell: int) -> None:
    """Form the dense practical-form Hessian H = X^T M_y X + beta M_u with
    X = A^{-1} M_yu at level ell-1 (the coarsest Hessian level, solved exactly
    as the theory of Section 3.2 assumes), symmetrise it and factor it.  Above
    dense_max rows no dense matrix is formed: that level is then solved by
    unpreconditioned CG to a loose tolerance, the practice of Section 5.2."""
    ell = max(1, min(ell, h.L))
    c = ell - 1
    n = h.levels[c].n
    h.ell = ell
    if n > h.opts.dense_max:
        h.H_dense = None
        h.chol_H = None
        return
    A, My, Mu, Myu = dense_level_matrices(h, c)
    X = sla.cho_solve(sla.cho_factor(A, lower=True), Myu)
    H = X.T @ (My @ X) + h.opts.beta * Mu
    H = 0.5 * (H + H.T)
    h.ell = ell
    h.H_dense = H
    h.chol_H = sla.cho_factor(H, lower=True)
