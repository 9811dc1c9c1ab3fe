"""Full-operator brute force for tiny circuits (n <= 8).

TEST INFRASTRUCTURE ONLY.

This is the evaluation the paper calls mathematically simple but wasteful
(Sec. 3, first paragraph): pad every gate to a 2^n x 2^n operator and
multiply the operators.  Two independent constructions are provided:

* `full_operator`: explicit entries, <i|U_full|j> = U[loc(i), loc(j)] when i
  and j agree on every bit outside the gate's qubits, else 0.
* `kron_operator`: Kronecker padding I (x) U (x) I for gates on adjacent,
  ascending qubits (little-endian: numpy's first Kronecker factor holds the
  most significant bits).

They are checked against each other in the tests, and the oracle's gate-by-
gate kernel is checked against them.
"""
from __future__ import annotations

import numpy as np

from . import gates as G


def _loc(idx: np.ndarray, qubits) -> np.ndarray:
    loc = np.zeros_like(idx)
    for t, q in enumerate(qubits):
        loc |= ((idx >> q) & 1) << t
    return loc


def full_operator(n: int, qubits, u: np.ndarray) -> np.ndarray:
    assert n <= 10
    idx = np.arange(1 << n, dtype=np.int64)
    mask = 0
    for q in qubits:
        mask |= 1 << q
    loc = _loc(idx, qubits)
    rest = idx & ~mask
    same = rest[:, None] == rest[None, :]
    return np.where(same, u[loc[:, None], loc[None, :]], 0.0).astype(np.complex128)


def kron_operator(n: int, qubits, u: np.ndarray) -> np.ndarray:
    qs = list(qubits)
    k = len(qs)
    assert qs == list(range(qs[0], qs[0] + k)), "adjacent ascending qubits only"
    lo = qs[0]
    hi = n - lo - k
    return np.kron(np.kron(np.eye(1 << hi), u), np.eye(1 << lo)).astype(np.complex128)


def circuit_operator(circ, params=None) -> np.ndarray:
    n = circ.n
    m = np.eye(1 << n, dtype=np.complex128)
    for g in circ.gates:
        th = g.theta if g.param < 0 else float(params[g.param])
        m = full_operator(n, g.qubits, G.matrix(g.op, th, g.mat)) @ m
    return m


def simulate(circ, params=None, psi0=None) -> np.ndarray:
    n = circ.n
    if psi0 is None:
        psi0 = np.zeros(1 << n, np.complex128)
        psi0[0] = 1.0
    return circuit_operator(circ, params) @ psi0


def pauli_matrix(n: int, x: int, z: int) -> np.ndarray:
    """i^{|x&z|} X^x Z^z as an explicit 2^n x 2^n matrix built per qubit by
    Kronecker products of 2x2 Pauli matrices (Y where both bits are set)."""
    m = np.ones((1, 1), np.complex128)
    for q in reversed(range(n)):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        p = G.I2 if not (bx or bz) else (G.X if bx and not bz else (G.Z if bz and not bx else G.Y))
        m = np.kron(m, p)
    return m
