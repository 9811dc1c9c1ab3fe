"""FP64 gate matrices for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Each matrix is written from its definition:
* H, NOT (X), Z, CNOT, CZ and T as printed in Sec. 2 (Background), with
  P = Z^(1/2) = diag(1, i) and the relations P = T^2, Z = T^4 of Sec. 4.3.
* sqrt(X), sqrt(Y), sqrt(W) as the principal square root of an involution G
  (G^2 = I): sqrt(G) = (1+i)/2 I + (1-i)/2 G.  For X this reproduces the
  matrix printed in Sec. 2; for Y the printed matrix differs (it squares to
  -Y), and the principal root is used (the configs name "sqrt(Y)").
  W = (X + Y)/sqrt(2).
* Rotations R_P(theta) = exp(-i theta P / 2); phase P(phi) = diag(1, e^{i phi});
  controlled phase CP(phi) = diag(1, 1, 1, e^{i phi}).
* Multi-qubit gates use the local index l = sum_t bit(q[t]) 2^t; CNOT has its
  control on q[0] and target on q[1] and is built from its action (flip the
  target when the control is 1), SWAP from its action (exchange the bits).
"""
from __future__ import annotations

import math

import numpy as np

C = math.sqrt(0.5)
OMEGA = complex(C, C)            # e^{i pi / 4}

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], np.complex128)
Y = np.array([[0, -1j], [1j, 0]], np.complex128)
Z = np.array([[1, 0], [0, -1]], np.complex128)
H = C * np.array([[1, 1], [1, -1]], np.complex128)
S = np.array([[1, 0], [0, 1j]], np.complex128)
T = np.array([[1, 0], [0, OMEGA]], np.complex128)
W = (X + Y) * C


def principal_sqrt_involution(g: np.ndarray) -> np.ndarray:
    return complex(0.5, 0.5) * np.eye(g.shape[0], dtype=np.complex128) + complex(0.5, -0.5) * g


SQRTX = principal_sqrt_involution(X)
SQRTY = principal_sqrt_involution(Y)
SQRTW = principal_sqrt_involution(W)


def by_action(k: int, fn) -> np.ndarray:
    """Permutation matrix of a k-qubit map on local indices: column l has a
    1 in row fn(l)."""
    d = 1 << k
    m = np.zeros((d, d), np.complex128)
    for l in range(d):
        m[fn(l), l] = 1.0
    return m


CNOT = by_action(2, lambda l: l ^ 2 if (l & 1) else l)       # control bit 0, target bit 1
SWAP = by_action(2, lambda l: ((l & 1) << 1) | ((l >> 1) & 1))
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)


def rx(t: float) -> np.ndarray:
    return math.cos(t / 2) * I2 - 1j * math.sin(t / 2) * X


def ry(t: float) -> np.ndarray:
    return math.cos(t / 2) * I2 - 1j * math.sin(t / 2) * Y


def rz(t: float) -> np.ndarray:
    return math.cos(t / 2) * I2 - 1j * math.sin(t / 2) * Z


def phase(t: float) -> np.ndarray:
    return np.array([[1, 0], [0, complex(math.cos(t), math.sin(t))]], np.complex128)


def cphase(t: float) -> np.ndarray:
    return np.diag([1, 1, 1, complex(math.cos(t), math.sin(t))]).astype(np.complex128)


FIXED = {
    "I": I2, "H": H, "X": X, "Y": Y, "Z": Z, "S": S, "SDG": S.conj().T,
    "T": T, "TDG": T.conj().T, "SQRTX": SQRTX, "SQRTY": SQRTY, "SQRTW": SQRTW,
    "SQRTXDG": SQRTX.conj().T, "SQRTYDG": SQRTY.conj().T, "SQRTWDG": SQRTW.conj().T,
    "CZ": CZ, "CNOT": CNOT, "SWAP": SWAP,
}
ANGLE = {"RX": rx, "RY": ry, "RZ": rz, "P": phase, "CP": cphase}
# Generator P of exp(-i theta P / 2) for the shift rule; P(phi) and CP(phi)
# equal such a rotation up to a global phase, so the same rule applies.
SHIFTABLE = {"RX", "RY", "RZ", "P", "CP"}


def matrix(op: str, theta: float = 0.0, mat: np.ndarray | None = None) -> np.ndarray:
    if op == "MAT":
        return np.asarray(mat, np.complex128)
    if op == "DIAG":                       # explicit diagonal entries
        return np.diag(np.asarray(mat, np.complex128).ravel())
    if op in FIXED:
        return FIXED[op]
    if op in ANGLE:
        return ANGLE[op](theta)
    raise KeyError(op)
