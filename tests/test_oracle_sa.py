"""Pins for the oracle's smoothed-aggregation hierarchy: brute-force
invariants of the aggregation, ordered-sum arithmetic checked against plain
Python loops, and the Galerkin identities of eqs. coarsestiffness/coarsemass."""
import numpy as np
import pytest

import inputs
from oracle import fem, sa
from oracle.csr import CSR, ordered_segment_sum, transpose


def _problem(kind):
    if kind == "2d":
        p = inputs.config("c1", n=12)
    elif kind == "2dj":
        p = inputs.config("c2", n=16)
    else:
        p = inputs.config("c3", n=5)
    A, M = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
    bc = p.dirichlet.astype(bool)
    return fem.dirichlet_stiffness(A, bc), M, bc, p


def test_splitmix64_published_vectors():
    # SplitMix64 seeded with 0 produces 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    # 0x06c45d188009454f (state advanced by the golden gamma before mixing).
    gamma = 0x9E3779B97F4A7C15
    x = np.array([0, gamma, (2 * gamma) % (1 << 64)], dtype=np.uint64)
    out = sa.splitmix64(x)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_ordered_segment_sum_is_left_to_right():
    rng = np.random.default_rng(0)
    lens = rng.integers(0, 9, size=50)
    ptr = np.concatenate([[0], np.cumsum(lens)])
    v = rng.standard_normal(ptr[-1]) * 10.0 ** rng.integers(-8, 8, size=ptr[-1])
    out = ordered_segment_sum(v, ptr)
    for s in range(50):
        acc = 0.0
        for p in range(ptr[s], ptr[s + 1]):
            acc = acc + float(v[p])
        assert out[s] == acc


@pytest.mark.parametrize("kind", ["2d", "2dj", "3d"])
def test_greedy_mis2_equals_parallel_rounds_and_is_maximal(kind):
    A0, M, bc, _ = _problem(kind)
    flags = sa.strength(A0, 0.08, bc)
    G = sa.strong_graph(A0, flags)
    keys = sa.priority_hash(A0.nrows, 0, inputs.AGG_SEED)
    root = sa.mis2_greedy(G, keys, ~bc)
    assert np.array_equal(root, sa.mis2_rounds(G, keys, ~bc))
    # brute-force distances in the strong graph
    n = A0.nrows
    adj = np.zeros((n, n), dtype=bool)
    adj[G.rows(), G.col] = True
    within2 = adj | (adj.astype(int) @ adj.astype(int) > 0) | np.eye(n, dtype=bool)
    R = np.nonzero(root)[0]
    sub = within2[np.ix_(R, R)]
    assert np.array_equal(sub, np.eye(R.size, dtype=bool))            # independent
    cover = within2[:, R].any(axis=1)
    assert np.all(cover[~bc])                                          # maximal
    assert not np.any(root[bc])


@pytest.mark.parametrize("kind", ["2d", "2dj", "3d"])
def test_aggregates_partition_and_are_connected(kind):
    A0, M, bc, _ = _problem(kind)
    flags = sa.strength(A0, 0.08, bc)
    G = sa.strong_graph(A0, flags)
    root = sa.mis2_greedy(G, sa.priority_hash(A0.nrows, 0, inputs.AGG_SEED), ~bc)
    agg, nc = sa.aggregate(A0, G, root, bc)
    assert np.all(agg[bc] == -1) and np.all(agg[~bc] >= 0)
    assert set(agg[~bc].tolist()) == set(range(nc))
    # coarse ids follow ascending root index
    assert np.array_equal(agg[np.nonzero(root)[0]], np.arange(nc))
    n = A0.nrows
    adj = [set() for _ in range(n)]
    for i, k in zip(G.rows(), G.col):
        adj[i].add(int(k))
    for J in range(nc):
        members = set(np.nonzero(agg == J)[0].tolist())
        start = int(np.nonzero(root & (agg == J))[0][0])
        seen, stack = {start}, [start]
        while stack:
            v = stack.pop()
            for w in adj[v]:
                if w in members and w not in seen:
                    seen.add(w)
                    stack.append(w)
        assert seen == members


def test_phase2_phase3_rules_brute_force():
    A0, M, bc, _ = _problem("2dj")
    flags = sa.strength(A0, 0.08, bc)
    G = sa.strong_graph(A0, flags)
    root = sa.mis2_greedy(G, sa.priority_hash(A0.nrows, 0, inputs.AGG_SEED), ~bc)
    agg, nc = sa.aggregate(A0, G, root, bc)
    n = A0.nrows
    nbr = {i: [] for i in range(n)}
    for i, k, v in zip(G.rows(), G.col, G.val):
        nbr[int(i)].append((int(k), abs(float(v))))
    cid = np.cumsum(root) - 1
    p2 = set()
    for i in range(n):
        if bc[i] or root[i]:
            continue
        rn = [(k, v) for k, v in nbr[i] if root[k]]
        if rn:
            best = max(rn, key=lambda t: (t[1], -t[0]))
            assert agg[i] == cid[best[0]]
            p2.add(i)
    for i in range(n):
        if bc[i] or root[i] or i in p2:
            continue
        cand = [(k, v) for k, v in nbr[i] if k in p2]
        best = max(cand, key=lambda t: (t[1], -t[0]))
        assert agg[i] == agg[best[0]]


def _loop_spgemm(A: CSR, B: CSR):
    out = {}
    for i in range(A.nrows):
        row = {}
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            k = A.col[p]
            for q in range(B.rowptr[k], B.rowptr[k + 1]):
                J = int(B.col[q])
                prod = float(A.val[p]) * float(B.val[q])
                row[J] = row.get(J, 0.0) + prod if J in row else 0.0 + prod
        for J, v in row.items():
            out[(i, J)] = v
    return out


def test_prolongator_and_galerkin_match_python_loops_bitwise():
    A0, M, bc, _ = _problem("2dj")
    flags = sa.strength(A0, 0.08, bc)
    G = sa.strong_graph(A0, flags)
    root = sa.mis2_greedy(G, sa.priority_hash(A0.nrows, 0, inputs.AGG_SEED), ~bc)
    agg, nc = sa.aggregate(A0, G, root, bc)
    S, omega, rho = sa.smooth_prolongator(A0, agg, nc, bc)
    d = A0.diag()
    # rho and omega by loops
    rr = 0.0
    for i in range(A0.nrows):
        if bc[i]:
            continue
        s = 0.0
        for p in range(A0.rowptr[i], A0.rowptr[i + 1]):
            s = s + abs(float(A0.val[p]))
        rr = max(rr, s / d[i])
    assert rho == rr and omega == (4.0 / 3.0) / rr
    for i in range(A0.nrows):
        ent = {}
        if not bc[i]:
            for p in range(A0.rowptr[i], A0.rowptr[i + 1]):
                J = agg[A0.col[p]]
                if J >= 0:
                    ent[J] = (ent[J] if J in ent else 0.0) + float(A0.val[p])
        cols = S.col[S.rowptr[i]:S.rowptr[i + 1]].tolist()
        assert cols == sorted(ent)
        for q, J in enumerate(cols):
            v = (omega * ent[J]) / d[i]
            ref = (1.0 if agg[i] == J else 0.0) - v
            assert S.val[S.rowptr[i] + q] == ref
    St = transpose(S)
    T = sa.spgemm_ordered(A0, S)
    ref_T = _loop_spgemm(A0, S)
    assert T.nnz == len(ref_T)
    for i, J, v in zip(T.rows(), T.col, T.val):
        assert ref_T[(int(i), int(J))] == v
    C = sa.spgemm_ordered(St, T)
    ref_C = _loop_spgemm(St, T)
    for i, J, v in zip(C.rows(), C.col, C.val):
        assert ref_C[(int(i), int(J))] == v
    # dense identities: S^T A S, exactly symmetric after mirroring
    Ac = sa.galerkin(S, St, A0)
    Sd = S.dense()
    np.testing.assert_allclose(Ac.dense(), Sd.T @ A0.dense() @ Sd, rtol=0, atol=1e-14 * np.abs(Ac.val).max())
    assert np.array_equal(Ac.dense(), Ac.dense().T)
    assert np.linalg.eigvalsh(Ac.dense()).min() > 0


def test_prolongator_preserves_constants_away_from_boundary():
    # kappa = 1: interior rows whose neighbours are all interior have zero row
    # sum, so (S 1)_i = 1 - omega (sum_k a_ik)/a_ii = 1 (partition of unity).
    A0, M, bc, p = _problem("2d")
    h = sa.build(A0, M, bc, sa.Opts(beta=p.beta, max_coarse=20))
    S = h.levels[0].S
    s1 = S.matvec(np.ones(S.ncols))
    rsum = A0.matvec(np.ones(A0.nrows))
    inner = (~bc) & (np.abs(rsum) < 1e-14)
    assert inner.sum() > 10
    assert np.max(np.abs(s1[inner] - 1.0)) < 1e-14


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_hierarchy_is_deterministic_and_spd(kind):
    A0, M, bc, p = _problem(kind)
    o = sa.Opts(beta=p.beta, max_coarse=20)
    h1 = sa.build(A0, M, bc, o)
    h2 = sa.build(A0, M, bc, o)
    assert h1.L >= 2
    for a, b in zip(h1.levels, h2.levels):
        assert np.array_equal(a.A.col, b.A.col) and np.array_equal(a.A.val, b.A.val)
        assert np.array_equal(a.M.val, b.M.val)
    for lev in h1.levels[1:]:
        Ad = lev.A.dense()
        assert np.array_equal(Ad, Ad.T)
        assert np.linalg.eigvalsh(Ad).min() > 0
        Md = lev.M.dense()
        assert np.linalg.eigvalsh(Md).min() > 0
    # coarse mass = S^T M S (eq. coarsemass with P = S)
    S = h1.levels[0].S.dense()
    np.testing.assert_allclose(h1.levels[1].M.dense(), S.T @ M.dense() @ S, rtol=0,
                               atol=1e-14 * np.abs(h1.levels[1].M.val).max())
