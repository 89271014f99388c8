"""Dense-matrix checker for QAOA on k-NAE-SAT (n <= 10), NumPy only.

TEST INFRASTRUCTURE, written independently of ``oracle.c`` to pin it: the cost
comes from the Pauli-Z (Walsh) expansion of the problem Hamiltonian, not from
evaluating literals, and the mixer is the matrix exponential of the dense
H_B = sum_j X_j, not a product of per-qubit passes.
"""
from __future__ import annotations

import itertools

import numpy as np

_X = np.array([[0.0, 1.0], [1.0, 0.0]])
_I2 = np.eye(2)


def z_values(n: int) -> np.ndarray:
    """z_v(x) = 1 - 2 x_v as an [n, 2^n] array, with x_v = bit v of x.

    Z_v acting on |x> gives z_v(x) |x> (Appendix A.1: the representing
    Hamiltonian of x_v is (I - Z_v)/2)."""
    x = np.arange(1 << n)
    return np.stack([1 - 2 * ((x >> v) & 1) for v in range(n)]).astype(np.float64)


def walsh_cost(clauses, n: int) -> np.ndarray:
    """Diagonal of H_C built from Pauli-Z products (Appendix A.2).

    A literal on variable v is represented by (I + s Z_v)/2 with s = -1 for a
    positive literal and s = +1 for a negated one (eq. repliteral). A clause is
    NAE-violated when all literals are false or all are true, so its
    Hamiltonian is H_{not sigma} + H_{all literals true}
      = 2^-k prod_j (I - s_j Z_j) + 2^-k prod_j (I + s_j Z_j),
    whose odd-order Z products cancel, leaving
      2^{1-k} sum_{S subset of [k], |S| even} prod_{j in S} s_j Z_{v_j}.
    The constant terms are kept here (the paper drops them because they only
    shift the cost), so the result equals the violated-clause count."""
    cl = np.asarray(clauses, dtype=np.int64)
    z = z_values(n)
    total = np.zeros(1 << n)
    for clause in cl:
        k = len(clause)
        s = np.where(clause > 0, -1.0, 1.0)
        v = np.abs(clause) - 1
        term = np.zeros(1 << n)
        for size in range(0, k + 1, 2):
            for S in itertools.combinations(range(k), size):
                prod = np.ones(1 << n)
                for j in S:
                    prod = prod * s[j] * z[v[j]]
                term += prod
        total += term * 2.0 ** (1 - k)
    return total


def walsh_cost_sat(clauses, n: int) -> np.ndarray:
    """Diagonal of the k-SAT cost from Pauli-Z products (Appendix A.2): an
    OR-clause is violated when every literal is false, so its Hamiltonian is
    H_{not sigma} = 2^-k prod_j (I - s_j Z_j)
      = 2^-k sum_{S subset of [k]} (-1)^{|S|} prod_{j in S} s_j Z_{v_j},
    with s as in walsh_cost (odd orders kept: no global-flip symmetry)."""
    cl = np.asarray(clauses, dtype=np.int64)
    z = z_values(n)
    total = np.zeros(1 << n)
    for clause in cl:
        k = len(clause)
        s = np.where(clause > 0, -1.0, 1.0)
        v = np.abs(clause) - 1
        term = np.zeros(1 << n)
        for size in range(0, k + 1):
            for S in itertools.combinations(range(k), size):
                prod = np.full(1 << n, (-1.0) ** size)
                for j in S:
                    prod = prod * s[j] * z[v[j]]
                term += prod
        total += term * 2.0 ** (-k)
    return total


def mixer_hamiltonian(n: int) -> np.ndarray:
    """H_B = sum_j X_j as a dense 2^n x 2^n matrix (Appendix A.3). Qubit j is
    bit j of the basis index, so X_j is the Kronecker product with X in the
    j-th factor counted from the least significant end."""
    H = np.zeros((1 << n, 1 << n))
    for j in range(n):
        op = np.array([[1.0]])
        for q in reversed(range(n)):
            op = np.kron(op, _X if q == j else _I2)
        H += op
    return H


def mixer_unitary(n: int, beta: float, _cache={}) -> np.ndarray:
    """U_B(beta) = expm(-i beta H_B), through the eigendecomposition of the
    real symmetric H_B (Section 2.1)."""
    if n not in _cache:
        _cache[n] = np.linalg.eigh(mixer_hamiltonian(n))
    w, V = _cache[n]
    return (V * np.exp(-1j * beta * w)) @ V.T


def qaoa_state(cost: np.ndarray, n: int, gammas, betas) -> np.ndarray:
    """prod_l U_B(beta_l) U_C(gamma_l) |+>, layer 0 first (Section 3.3), as
    dense matrix-vector products."""
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for g, b in zip(np.atleast_1d(gammas), np.atleast_1d(betas)):
        UC = np.diag(np.exp(-1j * g * np.asarray(cost, dtype=np.float64)))
        psi = mixer_unitary(n, b) @ (UC @ psi)
    return psi


def qaoa(cost: np.ndarray, n: int, gammas, betas):
    """(p_succ, E[C], norm): projector onto C = 0, <H_C> and <psi|psi>."""
    psi = qaoa_state(cost, n, gammas, betas)
    prob = np.abs(psi) ** 2
    c = np.asarray(cost, dtype=np.float64)
    return float(prob[c == 0].sum()), float((c * prob).sum()), float(prob.sum())
