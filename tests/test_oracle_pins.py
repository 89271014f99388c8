"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property it checks. None of them re-types the oracle's own
formula: the references are closed forms, invariants, special cases, a dense
construction from the Pauli-Z expansion with a matrix exponential, and brute
force written independently below.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import dense
from workloads import instances as inst


def rand_instance(n, k, m, seed):
    return inst.instance(n, k, m, seed)


# ---------------------------------------------------------------------------
# Brute force written from the definitions in plain Python (tiny n only)
# ---------------------------------------------------------------------------

def brute_cost(clauses, n):
    """NAE violated iff the literals are not (at least one true and at least
    one false): Section 2.2 and the Not-All-Equal condition."""
    out = []
    for x in range(1 << n):
        bits = [(x >> v) & 1 for v in range(n)]
        c = 0
        for cl in clauses:
            vals = [bits[abs(l) - 1] if l > 0 else 1 - bits[abs(l) - 1] for l in cl]
            if not (any(vals) and not all(vals)):
                c += 1
        out.append(c)
    return np.array(out)


def brute_qaoa(cost, n, gammas, betas):
    """Kronecker-product single-qubit rotations applied one qubit at a time,
    with complex Python numbers (no NumPy linear algebra)."""
    N = 1 << n
    psi = [complex(2 ** (-n / 2))] * N
    for g, b in zip(gammas, betas):
        psi = [psi[x] * complex(math.cos(g * cost[x]), -math.sin(g * cost[x])) for x in range(N)]
        R = [[math.cos(b), -1j * math.sin(b)], [-1j * math.sin(b), math.cos(b)]]
        for j in range(n):
            new = [0j] * N
            for x in range(N):
                bj = (x >> j) & 1
                for out_bit in (0, 1):
                    y = (x & ~(1 << j)) | (out_bit << j)
                    new[y] += R[out_bit][bj] * psi[x]
            psi = new
    prob = [abs(a) ** 2 for a in psi]
    return (sum(pr for pr, c in zip(prob, cost) if c == 0),
            sum(pr * c for pr, c in zip(prob, cost)), sum(prob))


@pytest.mark.parametrize("seed", range(6))
def test_cost_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 6))
    k = int(rng.integers(1, n + 1))
    m = int(rng.integers(0, 9))
    cl = rand_instance(n, k, m, seed).reshape(m, k)
    assert np.array_equal(oracle.cost(cl, n), brute_cost(cl, n))


@pytest.mark.parametrize("seed", range(4))
def test_qaoa_brute_force_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    n, k, m, p = 4, 3, 5, 3
    cl = rand_instance(n, k, m, seed)
    cost = brute_cost(cl, n)
    g, b = rng.uniform(-3, 3, p), rng.uniform(-3, 3, p)
    ref = brute_qaoa(list(cost), n, g, b)
    got = oracle.qaoa(cost, n, g, b)
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# P6: cost equals the Pauli-Z (Walsh) expansion of Appendix A.2
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("seed", range(3))
def test_cost_matches_walsh_expansion(k, seed):
    n = 9
    m = 4 * n
    cl = rand_instance(n, k, m, 10 * k + seed)
    assert np.array_equal(oracle.cost(cl, n), dense.walsh_cost(cl, n).round().astype(np.int64))
    assert np.allclose(dense.walsh_cost(cl, n), oracle.cost(cl, n), atol=1e-9)


def test_cost_repeated_variables_literal_by_literal():
    """A variable repeated with both signs always yields one true and one false
    literal, so such a clause never violates; a variable repeated with one
    sign behaves as the shorter clause."""
    n = 4
    cl = np.array([[1, -1, 2], [3, 3, -4], [2, 4, 4]], dtype=np.int32)
    c = oracle.cost(cl, n)
    assert np.array_equal(c, brute_cost(cl, n))
    assert np.array_equal(c, dense.walsh_cost(cl, n).round().astype(np.int64))


# ---------------------------------------------------------------------------
# P2, P3, P7: integer identities of the cost diagonal
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [2, 3, 5])
@pytest.mark.parametrize("n", [8, 13])
def test_cost_sum_closed_form(k, n):
    """Each clause with k distinct variables is violated on exactly 2 * 2^{n-k}
    assignments (Appendix B: probability 2^{1-k}), so sum_x C(x) = m 2^{n+1-k}."""
    m = 3 * n
    cl = rand_instance(n, k, m, n + k)
    assert int(oracle.cost(cl, n).sum()) == m * 2 ** (n + 1 - k)


@pytest.mark.parametrize("seed", range(4))
def test_cost_global_flip_symmetry(seed):
    """Z2 symmetry under the global bit flip (Section 2.2): C(x) = C(NOT x);
    solutions come in pairs."""
    n = 12
    cl = rand_instance(n, 3, 25, seed)
    c = oracle.cost(cl, n)
    x = np.arange(1 << n)
    assert np.array_equal(c, c[x ^ ((1 << n) - 1)])
    assert oracle.count_solutions(cl, n) % 2 == 0
    assert oracle.count_solutions(cl, n) == int((c == 0).sum())


def test_nae_equals_sat_of_x_and_complement():
    """Appendix A.5 lemma: x NAE-satisfies a clause iff x and its complement
    both satisfy it as an OR-clause."""
    n = 7
    cl = rand_instance(n, 3, 20, 5)
    c = oracle.cost(cl, n)
    full = (1 << n) - 1
    for x in range(1 << n):
        viol = 0
        for clause in cl:
            def sat(y):
                return any(((y >> (abs(l) - 1)) & 1) == (1 if l > 0 else 0) for l in clause)
            viol += 0 if (sat(x) and sat(x ^ full)) else 1
        assert viol == c[x]


# ---------------------------------------------------------------------------
# k-SAT predicate (Section 2.2: an OR-clause is violated iff all literals are
# false)
# ---------------------------------------------------------------------------

def brute_cost_sat(clauses, n):
    out = []
    for x in range(1 << n):
        c = 0
        for cl in clauses:
            if not any(((x >> (abs(l) - 1)) & 1) == (1 if l > 0 else 0) for l in cl):
                c += 1
        out.append(c)
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_sat_cost_brute_force_and_walsh(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 9))
    k = int(rng.integers(1, min(n, 5) + 1))
    m = int(rng.integers(0, 4 * n))
    cl = rand_instance(n, k, m, 70 + seed).reshape(m, k)
    c = oracle.cost(cl, n, "sat")
    assert np.array_equal(c, brute_cost_sat(cl, n))
    assert np.array_equal(c, dense.walsh_cost_sat(cl, n).round().astype(np.int64))
    assert oracle.count_solutions(cl, n, "sat") == int((c == 0).sum())
    xs = np.arange(0, 1 << n, 3, dtype=np.uint64)
    assert np.array_equal(oracle.cost_at(cl, n, xs, "sat"), c[xs.astype(np.int64)])


def test_sat_repeated_variables():
    """x OR NOT x is never violated; a repeated same-sign literal acts once."""
    cl = np.array([[1, -1, 2], [3, 3, -4], [-2, -2, -2]], dtype=np.int32)
    c = oracle.cost(cl, 4, "sat")
    assert np.array_equal(c, brute_cost_sat(cl, 4))
    assert np.array_equal(c, dense.walsh_cost_sat(cl, 4).round().astype(np.int64))


@pytest.mark.parametrize("k", [1, 3, 5])
def test_sat_cost_sum_and_nae_decomposition(k):
    """Each k-SAT clause with distinct variables is violated on 2^{n-k}
    assignments, so sum_x C = m 2^{n-k}; and a clause is NAE-violated exactly
    when it is SAT-violated at x or at NOT x (Appendix A.5), never both, so
    C_NAE(x) = C_SAT(x) + C_SAT(NOT x)."""
    n = 11
    cl = rand_instance(n, k, 3 * n, 900 + k)
    sat = oracle.cost(cl, n, "sat")
    assert int(sat.sum()) == 3 * n * 2 ** (n - k)
    x = np.arange(1 << n)
    assert np.array_equal(oracle.cost(cl, n), sat + sat[x ^ ((1 << n) - 1)])


def test_sat_qaoa_matches_dense():
    """The QAOA oracle on a cost without the global-flip symmetry."""
    n, p = 6, 3
    cl = rand_instance(n, 3, 14, 4)
    c = oracle.cost(cl, n, "sat")
    x = np.arange(1 << n)
    assert not np.array_equal(c, c[x ^ ((1 << n) - 1)])
    rng = np.random.default_rng(8)
    g, b = rng.uniform(-2, 2, p), rng.uniform(-2, 2, p)
    assert np.allclose(oracle.qaoa(c, n, g, b), dense.qaoa(c, n, g, b), rtol=0, atol=1e-12)
    psi = oracle.state(c, n, g, b)
    assert np.allclose(psi, dense.qaoa_state(c, n, g, b), rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# P8: dense matrix exponential at small n
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("seed", range(3))
def test_state_matches_dense_expm(k, seed):
    rng = np.random.default_rng(1000 + 7 * k + seed)
    n = 7
    p = 4
    cl = rand_instance(n, k, 2 * n, seed)
    cost = dense.walsh_cost(cl, n).round().astype(np.int32)
    g, b = rng.uniform(-np.pi, np.pi, p), rng.uniform(-np.pi, np.pi, p)
    ref = dense.qaoa_state(cost, n, g, b)
    got = oracle.state(cost, n, g, b)
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.allclose(oracle.qaoa(cost, n, g, b), dense.qaoa(cost, n, g, b), rtol=0, atol=1e-12)


def test_mixer_sign_is_observable():
    """The mixer's sign matters (p(g, -b) != p(g, b)), so the dense check above
    tells exp(-i b H_B) from exp(+i b H_B)."""
    n = 6
    cl = rand_instance(n, 3, 10, 1)
    cost = oracle.cost(cl, n)
    a = oracle.qaoa(cost, n, [0.4, 0.7], [0.3, 0.2])
    b = oracle.qaoa(cost, n, [0.4, 0.7], [-0.3, -0.2])
    assert abs(a[1] - b[1]) > 1e-3


# ---------------------------------------------------------------------------
# P1, P5: special cases of Appendix B and unitarity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["p0", "gamma0", "beta0"])
@pytest.mark.parametrize("k", [2, 3, 5])
def test_random_assignment_special_cases(case, k):
    """If p = 0, or every gamma is 0, or every beta is 0, the state stays |+>
    up to a phase (Appendix B), so p_succ = #solutions / 2^n and
    E[C] = m 2^{1-k} exactly."""
    n = 11
    m = 2 * n
    cl = rand_instance(n, k, m, 3 * k)
    cost = oracle.cost(cl, n)
    rng = np.random.default_rng(k)
    p = 5
    g, b = rng.uniform(-3, 3, p), rng.uniform(-3, 3, p)
    if case == "p0":
        g, b = [], []
    elif case == "gamma0":
        g = np.zeros(p)
    else:
        b = np.zeros(p)
    ps, e, norm = oracle.qaoa(cost, n, g, b)
    assert abs(ps - oracle.count_solutions(cl, n) / 2 ** n) < 1e-13
    assert abs(e - m * 2.0 ** (1 - k)) < 1e-11
    assert abs(norm - 1) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_norm_preserved(seed):
    rng = np.random.default_rng(seed)
    n, p = 14, 6
    cl = rand_instance(n, 3, 29, seed)
    cost = oracle.cost(cl, n)
    g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
    assert abs(oracle.qaoa(cost, n, g, b)[2] - 1) < 1e-12


# ---------------------------------------------------------------------------
# P4, P9, P12: symmetries, periodicities and layer plumbing
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 5])
def test_state_global_flip_symmetry(p):
    """C and |+> are invariant under the global flip and the flip commutes with
    the mixer, so psi(x) = psi(NOT x) after any number of layers."""
    n = 10
    cl = rand_instance(n, 3, 21, p)
    cost = oracle.cost(cl, n)
    rng = np.random.default_rng(p)
    psi = oracle.state(cost, n, rng.uniform(0, 3, p), rng.uniform(0, 3, p))
    x = np.arange(1 << n)
    assert np.max(np.abs(psi - psi[x ^ ((1 << n) - 1)])) < 1e-14


def test_periodicities():
    """gamma -> gamma + 2 pi (integer spectrum of H_C); beta -> beta + pi/2
    (R(b + pi/2) = -i X R(b) and the state is flip-symmetric); and
    (gamma, beta) -> (-gamma, -beta) (complex conjugation, real C and |+>)."""
    n, p = 9, 3
    cl = rand_instance(n, 3, 19, 2)
    cost = oracle.cost(cl, n)
    g = np.array([0.3, -0.8, 1.1])
    b = np.array([0.2, 0.9, -0.4])
    base = np.array(oracle.qaoa(cost, n, g, b))
    for gg, bb in [(g + 2 * np.pi * np.array([1, -1, 2]), b),
                   (g, b + np.pi / 2 * np.array([1, 3, -1])),
                   (-g, -b)]:
        assert np.allclose(oracle.qaoa(cost, n, gg, bb), base, rtol=0, atol=1e-12)


def test_zero_last_beta_truncates_circuit():
    """With beta_p = 0 the last phase only changes phases of basis states, so
    the readout equals that of the first p - 1 layers."""
    n, p = 12, 4
    cl = rand_instance(n, 3, 25, 9)
    cost = oracle.cost(cl, n)
    g, b = inst.ramp_angles(p)
    assert b[-1] == 0.0
    full = oracle.qaoa(cost, n, g, b)
    trunc = oracle.qaoa(cost, n, g[:-1], b[:-1])
    assert np.allclose(full, trunc, rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# P10: p = 1 closed form for k = 2 all-positive clauses (graph MaxCut mapping)
# ---------------------------------------------------------------------------

def maxcut_p1_edge(gamma, beta, du, dv, lam):
    """Expected cut indicator of edge (u, v) for depth-1 QAOA
    exp(-i beta sum X) exp(-i gamma C_cut)|+> (Wang, Hadfield, Jiang, Rieffel,
    Phys. Rev. A 97, 022304 (2018)); d = degree - 1, lam = common neighbours."""
    return (0.5 + 0.25 * math.sin(4 * beta) * math.sin(gamma) * (math.cos(gamma) ** du + math.cos(gamma) ** dv)
            - 0.25 * math.sin(2 * beta) ** 2 * math.cos(gamma) ** (du + dv - 2 * lam)
            * (1 - math.cos(2 * gamma) ** lam))


def graph_nae_expected_cost(edges, n, gamma, beta):
    """For clauses (x_u OR x_v), NAE-violation is x_u == x_v, i.e. the edge is
    uncut; C_NAE = m - C_cut, so exp(-i g C_NAE) = phase * exp(-i (-g) C_cut)
    and E[C_NAE] = sum_edges (1 - cut(-g, b))."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    tot = 0.0
    for u, v in edges:
        tot += 1 - maxcut_p1_edge(-gamma, beta, len(adj[u]) - 1, len(adj[v]) - 1, len(adj[u] & adj[v]))
    return tot


@pytest.mark.parametrize("n", [5, 8, 16])
def test_ring_p1_closed_form(n):
    edges = [(i, (i + 1) % n) for i in range(n)]
    cl = np.array([[u + 1, v + 1] for u, v in edges], dtype=np.int32)
    cost = oracle.cost(cl, n)
    for g, b in [(0.37, 0.21), (-1.1, 0.6), (2.0, -0.35)]:
        e = oracle.qaoa(cost, n, [g], [b])[1]
        assert abs(e - graph_nae_expected_cost(edges, n, g, b)) < 1e-11
        assert abs(e - n / 2 * (1 + 0.5 * math.sin(4 * b) * math.sin(2 * g))) < 1e-11


@pytest.mark.parametrize("seed", range(3))
def test_random_graph_p1_closed_form(seed):
    rng = np.random.default_rng(seed)
    n = 9
    edges = sorted({tuple(sorted(rng.choice(n, 2, replace=False))) for _ in range(16)})
    cl = np.array([[u + 1, v + 1] for u, v in edges], dtype=np.int32)
    cost = oracle.cost(cl, n)
    g, b = rng.uniform(-2, 2), rng.uniform(-1, 1)
    e = oracle.qaoa(cost, n, [g], [b])[1]
    assert abs(e - graph_nae_expected_cost(edges, n, g, b)) < 1e-11


# ---------------------------------------------------------------------------
# P11: statistics of the random model (Appendix B)
# ---------------------------------------------------------------------------

def test_solution_fraction_mean():
    """Over F_k(n, m) instances, E[#solutions / 2^n] = (1 - 2^{1-k})^m
    (Appendix B: clauses independent, each violated w.p. 2^{1-k})."""
    n, k, m = 10, 3, 12
    fr = [oracle.count_solutions(rand_instance(n, k, m, s), n) / 2 ** n for s in range(400)]
    mean, sem = np.mean(fr), np.std(fr) / math.sqrt(len(fr))
    assert abs(mean - (1 - 2.0 ** (1 - k)) ** m) < 4 * sem


# ---------------------------------------------------------------------------
# P13: gradient
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("w", [(1.0, 0.0), (0.0, 1.0), (0.7, -0.2)])
def test_adjoint_matches_finite_differences(w):
    rng = np.random.default_rng(5)
    n, p = 9, 4
    cl = rand_instance(n, 3, 19, 4)
    cost = oracle.cost(cl, n)
    g, b = rng.uniform(0, 2, p), rng.uniform(-1, 1, p)
    dg, db, out = oracle.qaoa_grad(cost, n, g, b, *w)
    fg, fb = oracle.finite_difference_grad(cost, n, g, b, *w, h=1e-4)
    scale = 1 + abs(w[1]) * 19
    assert np.max(np.abs(dg - fg)) < 1e-7 * scale
    assert np.max(np.abs(db - fb)) < 1e-7 * scale
    assert np.allclose(out, oracle.qaoa(cost, n, g, b), rtol=0, atol=1e-13)


def test_gradient_special_cases():
    """At beta = 0 every dF/dgamma vanishes, at gamma = 0 every dF/dbeta
    vanishes: the modulus of the state stays uniform."""
    n, p = 8, 3
    cl = rand_instance(n, 3, 17, 8)
    cost = oracle.cost(cl, n)
    dg, _, _ = oracle.qaoa_grad(cost, n, [0.3, 0.5, 0.9], [0, 0, 0], 1.0, 0.5)
    assert np.max(np.abs(dg)) < 1e-13
    _, db, _ = oracle.qaoa_grad(cost, n, [0, 0, 0], [0.3, 0.5, 0.9], 1.0, 0.5)
    assert np.max(np.abs(db)) < 1e-13


def test_gradient_matches_dense_finite_differences():
    """Finite differences of the dense construction, independent of the
    oracle's forward."""
    rng = np.random.default_rng(11)
    n, p = 6, 3
    cl = rand_instance(n, 3, 13, 11)
    cost = dense.walsh_cost(cl, n).round().astype(np.int32)
    g, b = rng.uniform(0, 2, p), rng.uniform(-1, 1, p)
    dg, db, _ = oracle.qaoa_grad(cost, n, g, b, 0.3, 1.0)
    h = 1e-5
    for i in range(p):
        e = np.zeros(p)
        e[i] = h
        def F(gg, bb):
            ps, en, _ = dense.qaoa(cost, n, gg, bb)
            return 0.3 * ps + en
        assert abs((F(g + e, b) - F(g - e, b)) / (2 * h) - dg[i]) < 1e-7
        assert abs((F(g, b + e) - F(g, b - e)) / (2 * h) - db[i]) < 1e-7


# ---------------------------------------------------------------------------
# Sampling bitstrings from the final state (Section 4.2: instance running time)
# ---------------------------------------------------------------------------

def brute_sample(psi, u):
    """Walk the outcomes in index order until the running mass passes u times
    the total (plain Python)."""
    probs = [abs(complex(a)) ** 2 for a in psi]
    total = sum(probs)
    out = []
    for uu in u:
        acc = 0.0
        for x, pr in enumerate(probs):
            acc += pr
            if acc > uu * total:
                out.append(x)
                break
    return out


@pytest.mark.parametrize("seed", range(3))
def test_sample_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 5
    cl = rand_instance(n, 3, 8, seed)
    psi = oracle.state(oracle.cost(cl, n), n, rng.uniform(0, 3, 2), rng.uniform(0, 3, 2))
    u = rng.random(300)
    assert list(oracle.sample(psi, n, u)) == brute_sample(psi, u)


def test_sample_uniform_state_closed_form():
    """|+> (p = 0): every outcome has mass 2^-n, so x = floor(u 2^n) away from
    the cell boundaries."""
    n = 16
    psi = oracle.state(np.zeros(1 << n, dtype=np.int32), n, [], [])
    rng = np.random.default_rng(1)
    u = rng.random(5000)
    frac = u * 2 ** n - np.floor(u * 2 ** n)
    u = u[(frac > 1e-6) & (frac < 1 - 1e-6)]
    assert np.array_equal(oracle.sample(psi, n, u), np.floor(u * 2 ** n).astype(np.uint64))


def test_sample_skips_zero_mass_and_normalises():
    psi = np.array([0, 0.6, 0, 0, 0.8j, 0, 0, 0], dtype=np.complex128) * 3.0  # norm 9
    s = oracle.sample(psi, 3, [0.0, 0.3599, 0.3601, 0.999999])
    assert list(s) == [1, 1, 4, 4]


def test_sample_frequencies_and_running_time():
    """Empirical frequencies match |psi|^2 (within 5 standard errors) and the
    mean running time matches the geometric mean 1/p_succ."""
    n, p = 6, 2
    cl = rand_instance(n, 3, 10, 3)
    c = oracle.cost(cl, n)
    g, b = [0.7, 0.4], [-0.5, -0.3]
    psi = oracle.state(c, n, g, b)
    prob = np.abs(psi) ** 2
    rng = np.random.default_rng(5)
    S = 400_000
    s = oracle.sample(psi, n, rng.random(S)).astype(np.int64)
    freq = np.bincount(s, minlength=1 << n) / S
    se = np.sqrt(prob * (1 - prob) / S)
    assert np.all(np.abs(freq - prob) <= 5 * se + 1e-12)
    ps = oracle.qaoa(c, n, g, b)[0]
    hits = np.flatnonzero(c[s] == 0)
    runs = np.diff(np.concatenate([[-1], hits]))  # i.i.d. running times
    assert oracle.running_time(s, c) == runs[0]
    assert oracle.running_time(s[hits[0] + 1:], c) == runs[1]
    assert oracle.running_time(s[c[s] > 0], c) == 0
    mean = np.mean(runs)
    assert abs(mean - 1 / ps) <= 5 * np.sqrt((1 - ps) / ps ** 2 / len(runs)), (mean, 1 / ps)


def test_oracle_threads_do_not_change_results():
    """The state update is elementwise, so any thread count gives the same
    state bit for bit; the readout sums differ only in rounding order."""
    cl = inst.instance(12, 3, 25, 3)
    c = oracle.cost(cl, 12)
    g, b = inst.ramp_angles(3)
    threads = oracle.num_threads()
    try:
        assert oracle.set_threads(1) == 1
        s1 = oracle.state(c, 12, g, b)
        r1 = oracle.qaoa(c, 12, g, b)
    finally:
        oracle.set_threads(threads)
    assert oracle.num_threads() == threads
    sn = oracle.state(c, 12, g, b)
    rn = oracle.qaoa(c, 12, g, b)
    assert np.array_equal(s1, sn)
    assert np.allclose(r1, rn, rtol=1e-13, atol=1e-16)


def test_stored_cost_digests():
    """The stored full-size diagonal digests against what the paper fixes:
    each clause of k distinct variables is violated on 2^(n+1-k) states
    under NAE (App. B) and on 2^(n-k) under k-SAT (Section 2.2), so the
    stored sums are m times that; the zero counts equal the stored
    workloads' solution counts and are even under NAE (global flip,
    Section 2.2); and the n = 24 digests equal a hash of the whole diagonal
    from the oracle's other entry point (the full-array routine)."""
    import hashlib
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "tests", "golden", "cost_digests.json")) as f:
        dig = json.load(f)
    with open(os.path.join(root, "tests", "golden", "workloads.json")) as f:
        work = json.load(f)
    assert set(dig) == set(inst.DIGEST_WORKLOADS)
    for name, rec in dig.items():
        n, k, m = rec["n"], rec["k"], rec["m"]
        assert (n, k, rec["r"], rec["predicate"]) == inst.DIGEST_WORKLOADS[name]
        assert m == inst.clause_count(n, rec["r"])
        assert rec["dtype"] == ("uint8" if m <= 255 else "uint16")
        per_clause = 2 ** (n + 1 - k) if rec["predicate"] == "nae" else 2 ** (n - k)
        assert rec["sum"] == m * per_clause, name
        assert len(rec["chunks"]) == 2 ** (n - rec["chunk_log2"])
        if rec["predicate"] == "nae":
            assert rec["num_zeros"] % 2 == 0
        if name in work:
            assert rec["seed"] == work[name]["seed"] and rec["num_zeros"] == work[name]["num_solutions"]
    rec = dig["nae3_n24_p10"]
    c = oracle.cost(inst.instance(24, 3, rec["m"], rec["seed"]), 24).astype(np.uint8).tobytes()
    assert hashlib.sha256(c).hexdigest() == rec["sha256"]
    assert hashlib.sha256(c).hexdigest()[:16] == rec["chunks"][0]
