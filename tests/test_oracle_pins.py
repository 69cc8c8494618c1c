"""Pins for the parts of the oracle's smoothed-aggregation setup that are
readings rather than formulas of the paper (Section 3.1 names smoothed
aggregation; the constants are this build's choices): the strength test, the
threshold schedule over the levels, the stop rules of the coarsening and the
composition of the aggregation priority hash.

Each pin is an independent plain statement of the rule (Python loops over
Python floats, hand-built matrices whose outcome is known in advance, a
scalar SplitMix64 over Python integers).  Every pin is also run against a
copy of the oracle with one mistake planted in it (a strict instead of a
non-strict comparison, a missed halving, a shifted stop rule, a different hash
composition), and must reject that copy."""
from __future__ import annotations

import inspect
import textwrap

import numpy as np
import pytest

import inputs
from oracle import fem, sa
from oracle.csr import CSR


# ---------------------------------------------------------------------------
# planting a mistake: a copy of one oracle function with one text substitution,
# compiled against a copy of the module's globals (so the real module is untouched)
def mutant(name: str, old: str | None = None, new: str | None = None, **overrides):
    """A copy of sa.<name>, optionally with the text old replaced by new; the
    copy's calls of other oracle functions go to overrides where given."""
    src = textwrap.dedent(inspect.getsource(getattr(sa, name)))
    if old is not None:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    ns = dict(vars(sa))
    ns.update(overrides)
    exec(compile(src, f"<copy of sa.{name}>", "exec"), ns)
    return ns[name]


def csr_from_dense(D: np.ndarray, keep_zero_pattern: np.ndarray | None = None) -> CSR:
    mask = D != 0 if keep_zero_pattern is None else keep_zero_pattern
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(D.shape[0] + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return CSR(np.cumsum(rowptr), cols.astype(np.int64), D[rows, cols].astype(np.float64), D.shape[1])


# ---------------------------------------------------------------------------
# strength: k != i strong iff neither node is Dirichlet and
# a_ik * a_ik >= (theta * theta) * (a_ii * a_kk), three IEEE roundings
def strength_loop(A: CSR, theta: float, dirichlet: np.ndarray) -> np.ndarray:
    diag = {}
    for i in range(A.nrows):
        for p in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
            if int(A.col[p]) == i:
                diag[i] = float(A.val[p])
    t = float(theta) * float(theta)
    out = np.zeros(A.nnz, dtype=bool)
    for i in range(A.nrows):
        for p in range(int(A.rowptr[i]), int(A.rowptr[i + 1])):
            k = int(A.col[p])
            if k == i or dirichlet[i] or dirichlet[k]:
                continue
            a = float(A.val[p])
            out[p] = a * a >= t * (diag.get(i, 0.0) * diag.get(k, 0.0))
    return out


def _tie_matrix():
    # rows with an exact tie a_ik^2 == theta^2 a_ii a_kk at theta = 0.5, an
    # explicit zero coupling, and a coupling just below the threshold
    D = np.array([[4.0, -2.0, 0.0, 0.0],
                  [-2.0, 4.0, -1.0, 0.0],
                  [0.0, -1.0, 4.0, -1.9999999999999998],
                  [0.0, 0.0, -1.9999999999999998, 4.0]])
    pattern = np.array([[1, 1, 1, 0], [1, 1, 1, 0], [1, 1, 1, 1], [0, 0, 1, 1]], dtype=bool)
    return csr_from_dense(D, pattern)


def strength_cases():
    cases = []
    for name, n in (("c1", 12), ("c2", 16)):
        p = inputs.config(name, n=n)
        A, _ = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
        bc = p.dirichlet.astype(bool)
        # the raw stiffness (couplings to Dirichlet nodes present) and the
        # Dirichlet-reduced one the hierarchy is built from
        cases += [(A, 0.08, bc), (fem.dirichlet_stiffness(A, bc), 0.08, bc), (A, 0.0, bc)]
    p = inputs.config("c3", n=5)
    A, _ = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
    bc = p.dirichlet.astype(bool)
    cases += [(A, 0.08, bc), (A, 0.02, bc), (fem.dirichlet_stiffness(A, bc), 0.04, bc)]
    T = _tie_matrix()
    cases += [(T, 0.5, np.zeros(4, dtype=bool)), (T, 0.5, np.array([False, False, False, True]))]
    return cases


def check_strength(fn) -> list:
    bad = []
    for ci, (A, theta, bc) in enumerate(strength_cases()):
        got = np.asarray(fn(A, theta, bc), dtype=bool)
        if not np.array_equal(got, strength_loop(A, theta, bc)):
            bad.append(ci)
    return bad


def test_strength_loop_sees_ties_zeros_and_dirichlet():
    # the loop itself on the hand-built case: the tie is strong, the explicit
    # zero and the coupling one ulp below the threshold are not, and a
    # Dirichlet node has no strong coupling
    T = _tie_matrix()
    f = strength_loop(T, 0.5, np.zeros(4, dtype=bool))
    flags = {(int(i), int(k)): bool(v) for i, k, v in zip(T.rows(), T.col, f)}
    assert flags[(0, 1)] and flags[(1, 0)]
    assert not flags[(0, 2)] and not flags[(2, 0)]          # explicit zero
    assert not flags[(1, 2)]                                 # 1 < 0.25 * 16
    assert not flags[(2, 3)]                                 # just below the tie
    f = strength_loop(T, 0.5, np.array([False, True, False, False]))
    touches = (T.rows() == 1) | (T.col == 1)
    assert not f[touches].any() and f.sum() == 0             # the tie was node 1's only strong pair


def test_strength_matches_loop():
    assert check_strength(sa.strength) == []


@pytest.mark.parametrize("old,new", [
    ("(lhs >= rhs)", "(lhs > rhs)"),                          # tie broken the other way
    ("~dirichlet[A.col] & ", ""),                             # Dirichlet neighbour not excluded
    ("(r != A.col) & ", ""),                                  # diagonal counted as a coupling
    ("lhs = aik * aik", "lhs = np.abs(aik)"),                 # not the squared test
    ("t = theta * theta", "t = theta"),                       # threshold not squared
])
def test_strength_pin_rejects_planted_mistakes(old, new):
    assert check_strength(mutant("strength", old, new)) != []


# ---------------------------------------------------------------------------
# threshold schedule theta_j = theta_0 / 2^j at every level the build visits
def thetas_seen(sub, theta0: float) -> tuple:
    seen = []

    def rec(A, theta, dirichlet):
        seen.append(theta)
        return sa.strength(A, theta, dirichlet)

    p = inputs.config("c1", n=32)
    A, M = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
    bc = p.dirichlet.astype(bool)
    build = mutant("build", *sub, strength=rec)
    h = build(fem.dirichlet_stiffness(A, bc), M, bc, sa.Opts(beta=1e-2, max_coarse=4, theta0=theta0))
    return seen, h.L


def check_theta_schedule(sub=(None, None)) -> bool:
    s1, L1 = thetas_seen(sub, 0.08)
    s2, _ = thetas_seen(sub, 0.2)
    return (len(s1) >= 3 and L1 == len(s1) + 1
            and s1 == [0.08, 0.04, 0.02, 0.01, 0.005, 0.0025][:len(s1)]
            and s2[:3] == [0.2, 0.1, 0.05])


def test_theta_schedule_halves_per_level():
    assert check_theta_schedule()


@pytest.mark.parametrize("old,new", [
    ("theta = opts.theta0 * 0.5 ** j", "theta = opts.theta0"),            # missed halving
    ("theta = opts.theta0 * 0.5 ** j", "theta = opts.theta0 * 0.5 ** (j + 1)"),
    ("theta = opts.theta0 * 0.5 ** j", "theta = 0.08 * 0.5 ** j"),        # option ignored
])
def test_theta_pin_rejects_planted_mistakes(old, new):
    assert not check_theta_schedule((old, new))


# ---------------------------------------------------------------------------
# stop rules: level j is the coarsest when n_j <= max_coarse, when j + 1 =
# max_levels, or when the aggregation would give n_{j+1} = 0 or > 0.9 n_j
def pairs_matrix(n: int, npairs: int):
    """n nodes, the first npairs pairs coupled by -1 (strong at any threshold
    below 1/2), the others isolated: the aggregation gives n - npairs
    aggregates (one per pair, one per isolated node)."""
    D = 2.0 * np.eye(n)
    for q in range(npairs):
        D[2 * q, 2 * q + 1] = D[2 * q + 1, 2 * q] = -1.0
    return csr_from_dense(D), csr_from_dense(np.eye(n) / n)


def levels_of(build_fn, A, M, bc, **kw) -> list:
    h = build_fn(A, M, bc, sa.Opts(beta=1e-2, **kw))
    return [lev.n for lev in h.levels]


def check_stop_rules(build_fn) -> list:
    bad = []
    # coarsening ratio: 10 -> 9 aggregates is not above 0.9 n, 20 -> 19 and
    # 10 -> 10 are
    A, M = pairs_matrix(10, 1)
    if levels_of(build_fn, A, M, np.zeros(10, bool), max_coarse=1, max_levels=2) != [10, 9]:
        bad.append("ratio 9/10")
    A, M = pairs_matrix(20, 1)
    if levels_of(build_fn, A, M, np.zeros(20, bool), max_coarse=1, max_levels=2) != [20]:
        bad.append("ratio 19/20")
    A, M = pairs_matrix(10, 0)
    if levels_of(build_fn, A, M, np.zeros(10, bool), max_coarse=1, max_levels=5) != [10]:
        bad.append("no coupling")
    # every node Dirichlet: no aggregate at all
    A, M = pairs_matrix(6, 0)
    try:
        if levels_of(build_fn, A, M, np.ones(6, bool), max_coarse=1) != [6]:
            bad.append("empty aggregation")
    except Exception:
        bad.append("empty aggregation raised")
    # max_coarse: a level of exactly max_coarse rows is the coarsest
    p = inputs.config("c1", n=12)
    Af, Mf = fem.assemble(p.mesh.coords, p.mesh.elems, p.kappa)
    bc = p.dirichlet.astype(bool)
    A0 = fem.dirichlet_stiffness(Af, bc)
    full = levels_of(build_fn, A0, Mf, bc, max_coarse=1)
    if len(full) < 3:
        bad.append("too few levels to test")
        return bad
    n0, n1 = full[0], full[1]
    if levels_of(build_fn, A0, Mf, bc, max_coarse=n0) != [n0]:
        bad.append("max_coarse = n0")
    if levels_of(build_fn, A0, Mf, bc, max_coarse=n1) != [n0, n1]:
        bad.append("max_coarse = n1")
    if len(levels_of(build_fn, A0, Mf, bc, max_coarse=n1 - 1)) < 3:
        bad.append("max_coarse = n1 - 1")
    # max_levels
    for m in (1, 2, 3):
        if len(levels_of(build_fn, A0, Mf, bc, max_coarse=1, max_levels=m)) != m:
            bad.append(f"max_levels = {m}")
    return bad


def test_stop_rules():
    assert check_stop_rules(sa.build) == []


@pytest.mark.parametrize("old,new", [
    ("nc > 0.9 * lev.n", "nc >= 0.9 * lev.n"),
    ("nc > 0.9 * lev.n", "nc > 0.95 * lev.n"),
    ("nc == 0 or ", ""),
    ("lev.n <= opts.max_coarse", "lev.n < opts.max_coarse"),
    ("j + 1 >= opts.max_levels", "j + 1 > opts.max_levels"),
])
def test_stop_pin_rejects_planted_mistakes(old, new):
    assert check_stop_rules(mutant("build", old, new)) != []


# ---------------------------------------------------------------------------
# aggregation priority: key(i) at level j = SplitMix64(seed ^ (j << 40) ^ i)
M64 = (1 << 64) - 1


def splitmix64_scalar(x: int) -> int:
    """SplitMix64's output function on one 64-bit word (Steele, Lea and Flood,
    OOPSLA 2014), over Python integers."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_scalar_splitmix64_published_vectors():
    # the generator seeded with 0: its state advances by the golden gamma before
    # each output
    gamma = 0x9E3779B97F4A7C15
    outs = [splitmix64_scalar((k * gamma) & M64) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def check_priority_hash(fn) -> list:
    bad = []
    for seed in (inputs.AGG_SEED, 0, (1 << 63) + 5, M64):
        for j in (0, 1, 2, 5):
            n = 3000
            got = fn(n, j, seed)
            for i in (0, 1, 2, 7, 255, 256, 1023, 2999):
                if int(got[i]) != splitmix64_scalar(seed ^ (j << 40) ^ i):
                    bad.append((seed, j, i))
    return bad


def test_priority_hash_composition():
    assert check_priority_hash(sa.priority_hash) == []


@pytest.mark.parametrize("old,new", [
    ("(level << 40)", "(level << 32)"),
    ("base ^ np.arange(n, dtype=U64)", "base + np.arange(n, dtype=U64)"),
    ("U64((seed ^ (level << 40)) & _M64)", "U64((seed ^ level) & _M64)"),
])
def test_hash_pin_rejects_planted_mistakes(old, new):
    assert check_priority_hash(mutant("priority_hash", old, new)) != []
