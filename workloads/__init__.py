"""Seeded synthetic inputs for the state-vector sweep.

This module only *describes* inputs: gate lists (names, qubit tuples,
parameter slots), parameter values drawn from a seeded generator, Pauli-sum
observables as (coefficient, x-mask, z-mask) triples, and random initial
states.  It holds no gate matrices and none of the simulation arithmetic, so
the CPU oracle and the GPU path can both consume it without sharing any of
the method.

Conventions
-----------
* Qubit ``q`` is bit ``q`` of the amplitude index (little-endian).  The paper
  reads qubit ``i_0`` as "bit position i_0" of the index (Sec. 4.3, the CZ and
  T bitmask discussion) and its bitmask examples (Fig. reorder) put the gate on
  qubit 0 in the least significant bit.
* Multi-qubit gates list their qubits in the order of the local matrix index:
  ``qubits[0]`` is the least significant bit of the gate's local index.  For
  ``CNOT`` that means ``qubits[0]`` is the control and ``qubits[1]`` the
  target, matching the matrix printed in Sec. 2.
* A parameterised gate carries ``param >= 0`` (an index into the parameter
  vector); otherwise ``theta`` holds its fixed angle.

The grid circuits stand in for the Google "v2" supremacy benchmarks the paper
measures on (Sec. 6): planar grid, an initial Hadamard layer, one random gate
from the sqrt(X)/sqrt(Y)/sqrt(W)/T family per qubit per cycle, and CZ gates on
one of four grid-edge patterns per cycle.  The benchmark files themselves are
not used or reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Gate vocabulary (names only).  Arity is part of the vocabulary, not of the
# arithmetic.
ARITY: Dict[str, int] = {
    "I": 1, "H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "SDG": 1, "T": 1, "TDG": 1,
    "SQRTX": 1, "SQRTY": 1, "SQRTW": 1, "SQRTXDG": 1, "SQRTYDG": 1, "SQRTWDG": 1,
    "RX": 1, "RY": 1, "RZ": 1, "P": 1,
    "CZ": 2, "CNOT": 2, "SWAP": 2, "CP": 2,
}
PARAMETRIC = {"RX", "RY", "RZ", "P", "CP"}
# Name of each gate's inverse (angle gates invert by negating the angle).
INVERSE_NAME = {"I": "I", "H": "H", "X": "X", "Y": "Y", "Z": "Z", "S": "SDG", "SDG": "S",
                "T": "TDG", "TDG": "T", "SQRTX": "SQRTXDG", "SQRTXDG": "SQRTX",
                "SQRTY": "SQRTYDG", "SQRTYDG": "SQRTY", "SQRTW": "SQRTWDG", "SQRTWDG": "SQRTW",
                "CZ": "CZ", "CNOT": "CNOT", "SWAP": "SWAP"}


@dataclass(frozen=True)
class Gate:
    op: str
    qubits: Tuple[int, ...]
    param: int = -1            # index into the parameter vector, or -1
    theta: float = 0.0         # fixed angle when param < 0
    mat: Optional[np.ndarray] = None  # explicit 2^k x 2^k complex matrix for op "MAT",
                                      # or the 2^k diagonal entries for op "DIAG"


@dataclass
class Circuit:
    n: int
    gates: List[Gate] = field(default_factory=list)
    n_params: int = 0
    name: str = ""

    def __len__(self) -> int:
        return len(self.gates)

    def cut(self, keep: int) -> "Circuit":
        """Sub-circuit on qubits [0, keep): only gates entirely inside are kept."""
        g = [x for x in self.gates if max(x.qubits) < keep]
        return Circuit(keep, g, self.n_params, f"{self.name}[cut{keep}]")

    def inverse_ops_available(self) -> bool:
        return all(x.op != "MAT" for x in self.gates)


@dataclass
class PauliSum:
    """Observable sum_k c_k * P_k with P_k = i^{|x_k & z_k|} X^{x_k} Z^{z_k}."""
    coeff: np.ndarray    # float64 [K]
    x_mask: np.ndarray   # uint64 [K]
    z_mask: np.ndarray   # uint64 [K]

    def __len__(self) -> int:
        return int(self.coeff.shape[0])


def pauli_sum(terms: Sequence[Tuple[float, Dict[int, str]]]) -> PauliSum:
    """Build a PauliSum from [(coeff, {qubit: 'X'|'Y'|'Z'})]."""
    c, xs, zs = [], [], []
    for coeff, ops in terms:
        x = z = 0
        for q, p in ops.items():
            if p in ("X", "Y"):
                x |= 1 << q
            if p in ("Z", "Y"):
                z |= 1 << q
        c.append(float(coeff))
        xs.append(x)
        zs.append(z)
    return PauliSum(np.array(c, np.float64), np.array(xs, np.uint64), np.array(zs, np.uint64))


# ----------------------------------------------------------------------------
# Generators
# ----------------------------------------------------------------------------

def line_circuit(n: int = 12, layers: int = 10, seed: int = 1000) -> Circuit:
    """Line of n qubits; each layer: a uniform gate from {H, sqrt(X), sqrt(Y), T}
    on every qubit, then CZ on (0,1),(2,3),... (even layers) or (1,2),(3,4),...
    (odd layers).  n=12, 10 layers gives 175 gates."""
    rng = np.random.default_rng(seed)
    fam = ["H", "SQRTX", "SQRTY", "T"]
    gates: List[Gate] = []
    for layer in range(layers):
        picks = rng.integers(0, 4, size=n)
        for q in range(n):
            gates.append(Gate(fam[int(picks[q])], (q,)))
        for a in range(layer % 2, n - 1, 2):
            gates.append(Gate("CZ", (a, a + 1)))
    return Circuit(n, gates, 0, f"line{n}x{layers}")


def grid_edges(rows: int, cols: int, pattern: str) -> List[Tuple[int, int]]:
    """CZ edge patterns on a row-major rows x cols grid (q = r*cols + c):
    A horizontal edges with c even, B horizontal with c odd,
    C vertical edges with r even, D vertical with r odd."""
    e = []
    if pattern in "AB":
        par = 0 if pattern == "A" else 1
        for r in range(rows):
            for c in range(par, cols - 1, 2):
                e.append((r * cols + c, r * cols + c + 1))
    else:
        par = 0 if pattern == "C" else 1
        for r in range(par, rows - 1, 2):
            for c in range(cols):
                e.append((r * cols + c, (r + 1) * cols + c))
    return e


def grid_circuit(rows: int, cols: int, cycles: int, seed: int,
                 family: Sequence[str] = ("SQRTX", "SQRTY", "SQRTW", "T"),
                 initial_h: bool = True) -> Circuit:
    """Random grid circuit: initial H layer, then `cycles` cycles of
    (i.i.d. uniform gate from `family` on every qubit; CZ on pattern
    [A, C, B, D][t mod 4])."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    gates: List[Gate] = []
    if initial_h:
        gates += [Gate("H", (q,)) for q in range(n)]
    order = "ACBD"
    for t in range(cycles):
        picks = rng.integers(0, len(family), size=n)
        for q in range(n):
            gates.append(Gate(family[int(picks[q])], (q,)))
        for a, b in grid_edges(rows, cols, order[t % 4]):
            gates.append(Gate("CZ", (a, b)))
    return Circuit(n, gates, 0, f"grid{rows}x{cols}x{cycles}")


def grid30(seed: int = 1001) -> Circuit:
    """30-qubit 5x6 grid, 20 cycles (875 gates)."""
    return grid_circuit(5, 6, 20, seed)


def grid33(seed: int = 1002, cycles: int = 40) -> Circuit:
    """33-qubit 3x11 grid, 40 cycles (1873 gates)."""
    return grid_circuit(3, 11, cycles, seed)


def ansatz_circuit(n: int = 20, layers: int = 10) -> Circuit:
    """Hardware-efficient ansatz: per layer RY(theta) then RZ(theta') on every
    qubit, then a CZ ladder (i, i+1), i = 0..n-2.  n=20, 10 layers: 590 gates,
    400 parameters."""
    gates: List[Gate] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("RY", (q,), param=p)); p += 1
            gates.append(Gate("RZ", (q,), param=p)); p += 1
        for a in range(n - 1):
            gates.append(Gate("CZ", (a, a + 1)))
    return Circuit(n, gates, p, f"ansatz{n}x{layers}")


def ansatz_observable(n: int = 20) -> PauliSum:
    """H = sum_{i=0}^{n-2} Z_i Z_{i+1} + 0.5 sum_{i=0}^{n-1} X_i (open chain)."""
    terms = [(1.0, {i: "Z", i + 1: "Z"}) for i in range(n - 1)]
    terms += [(0.5, {i: "X"}) for i in range(n)]
    return pauli_sum(terms)


def z_sum(n: int) -> PauliSum:
    return pauli_sum([(1.0, {i: "Z"}) for i in range(n)])


def uniform_params(count: int, n_params: int, seed: int) -> np.ndarray:
    """Angles ~ U[0, 2*pi), shape [count, n_params]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, size=(count, n_params))


def layered_param_circuit(n: int, layers: int, seed: int) -> Circuit:
    """Per layer: a random fixed gate from {H, sqrt(X), sqrt(Y), T} on every
    qubit, then RY(theta) on every qubit, then CZ on alternating neighbour
    pairs ((0,1),(2,3),... on even layers, (1,2),... on odd layers)."""
    rng = np.random.default_rng(seed)
    fam = ["H", "SQRTX", "SQRTY", "T"]
    gates: List[Gate] = []
    p = 0
    for layer in range(layers):
        picks = rng.integers(0, 4, size=n)
        for q in range(n):
            gates.append(Gate(fam[int(picks[q])], (q,)))
        for q in range(n):
            gates.append(Gate("RY", (q,), param=p)); p += 1
        for a in range(layer % 2, n - 1, 2):
            gates.append(Gate("CZ", (a, a + 1)))
    return Circuit(n, gates, p, f"layered{n}x{layers}")


def batch_circuits(count: int = 512, n_lo: int = 10, n_hi: int = 22,
                   l_lo: int = 20, l_hi: int = 60, seed0: int = 4000) -> List[Circuit]:
    """Many circuits with uneven qubit counts n ~ U{n_lo..n_hi} and
    L ~ U{l_lo..l_hi} layers; circuit i uses seed seed0 + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.integers(n_lo, n_hi + 1))
        layers = int(rng.integers(l_lo, l_hi + 1))
        out.append(layered_param_circuit(n, layers, seed0 + i))
    return out


def random_circuit(n: int, n_gates: int, seed: int,
                   ops: Sequence[str] = ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SQRTX",
                                         "SQRTY", "SQRTW", "RX", "RY", "RZ", "P", "CZ", "CNOT",
                                         "SWAP", "CP"),
                   mat_k: Sequence[int] = (), param_frac: float = 0.5,
                   diag_k: Sequence[int] = ()) -> Circuit:
    """Random circuit over `ops` with random (non-adjacent, any order) qubits.
    Angle gates get a parameter slot with probability `param_frac`, otherwise
    a fixed angle.  `mat_k` lists arities of random explicit-matrix gates to
    mix in (the matrices are Haar-ish random unitaries from a QR of a complex
    Gaussian, drawn here as input data); `diag_k` arities of explicit
    diagonal gates with random unit-modulus entries."""
    rng = np.random.default_rng(seed)
    choices = list(ops) + [f"MAT{k}" for k in mat_k] + [f"DIAG{k}" for k in diag_k]
    gates: List[Gate] = []
    p = 0
    for _ in range(n_gates):
        op = choices[int(rng.integers(0, len(choices)))]
        if op.startswith("DIAG"):
            k = int(op[4:])
            if k > n:
                continue
            qs = tuple(int(x) for x in rng.permutation(n)[:k])
            gates.append(Gate("DIAG", qs, mat=np.exp(1j * rng.uniform(-np.pi, np.pi, 1 << k))))
            continue
        if op.startswith("MAT"):
            k = int(op[3:])
            if k > n:
                continue
            qs = tuple(int(x) for x in rng.permutation(n)[:k])
            z = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
            qm, r = np.linalg.qr(z)
            qm = qm * (np.diag(r) / np.abs(np.diag(r)))
            gates.append(Gate("MAT", qs, mat=qm.astype(np.complex128)))
            continue
        k = ARITY[op]
        if k > n:
            continue
        qs = tuple(int(x) for x in rng.permutation(n)[:k])
        if op in PARAMETRIC:
            if rng.random() < param_frac:
                gates.append(Gate(op, qs, param=p)); p += 1
            else:
                gates.append(Gate(op, qs, theta=float(rng.uniform(-np.pi, np.pi))))
        else:
            gates.append(Gate(op, qs))
    return Circuit(n, gates, p, f"random{n}x{n_gates}s{seed}")


def inverse(c: Circuit) -> Circuit:
    """The mirror circuit U^dagger as a gate list: reversed order, each gate
    replaced by its inverse by name (fixed-angle gates negate the angle)."""
    out: List[Gate] = []
    for g in reversed(c.gates):
        if g.op in PARAMETRIC:
            if g.param >= 0:
                raise ValueError("inverse() needs fixed angles")
            out.append(Gate(g.op, g.qubits, -1, -g.theta))
        elif g.op in INVERSE_NAME:
            out.append(Gate(INVERSE_NAME[g.op], g.qubits))
        else:
            raise ValueError(f"no named inverse for {g.op}")
    return Circuit(c.n, out, 0, c.name + "^-1")


def concat(a: Circuit, b: Circuit) -> Circuit:
    assert a.n == b.n
    return Circuit(a.n, list(a.gates) + list(b.gates), max(a.n_params, b.n_params),
                   a.name + "+" + b.name)


def random_state(n: int, seed: int, batch: int = 0) -> np.ndarray:
    """Complex Gaussian state normalised to unit 2-norm (complex128).
    batch > 0 gives shape [batch, 2^n]."""
    rng = np.random.default_rng(seed)
    shape = (batch, 1 << n) if batch else (1 << n,)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    return v.astype(np.complex128)


def basis_state(n: int, index: int) -> np.ndarray:
    v = np.zeros(1 << n, np.complex128)
    v[index] = 1.0
    return v


def sample_uniforms(count: int, seed: int, batch: int = 0) -> np.ndarray:
    """Random numbers in [0, 1) that drive measurement sampling (float64).
    batch > 0 gives shape [batch, count]."""
    rng = np.random.default_rng(seed)
    return rng.random((batch, count) if batch else (count,))
