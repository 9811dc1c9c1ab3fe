"""FP64 CPU oracle for Schroedinger-style state-vector simulation.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library: it has its own gate table (oracle/gates.py), its own generic gate
kernel in plain C (oracle/sv_oracle.c, OpenMP over set ids) and its own
reductions.  It consumes the same seeded gate lists (package `workloads`).

What it computes (Sec. 3, "Fast Schroedinger simulation"): psi_out =
U_G ... U_2 U_1 psi_in, one gate at a time, each gate applied to every one of
the 2^{n-k} disjoint index sets of 2^k amplitudes.

Functions:
  simulate      gate-by-gate sweep in FP64
  expect        sum_k c_k <psi|P_k|psi> for a Pauli sum, compensated sums
  norm2         ||psi||^2 with Sum2 compensated summation (Sec. 4.1 norm check)
  energy        expect(simulate(...))
  grad_param_shift  exact gradient for exp(-i theta P/2) gates (two-term shift)
  grad_fd       central finite differences
  sample        measurement of all qubits by inverse-CDF sampling

Parity status: every function here is pinned by tests under tests/ (brute
force operator products, closed forms, printed matrices and identities of the
paper, exact summation); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import gates as G

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sv_oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C core with gcc (OpenMP, portable x86-64-v3 code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.or_apply.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp, ctypes.c_int]
        lib.or_apply.restype = ctypes.c_int
        lib.or_norm2.argtypes = [ctypes.c_int, dp, ctypes.c_int]
        lib.or_norm2.restype = ctypes.c_double
        lib.or_pauli_expect.argtypes = [ctypes.c_int, dp, ctypes.c_uint64, ctypes.c_uint64,
                                        dp, dp, ctypes.c_int]
        lib.or_inner.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
        lib.or_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().or_max_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gate_matrix(g, params: Optional[np.ndarray]) -> np.ndarray:
    theta = g.theta
    if g.param >= 0:
        theta = float(params[g.param])
    return G.matrix(g.op, theta, g.mat)


def apply_matrix(psi: np.ndarray, n: int, qubits: Sequence[int], u: np.ndarray,
                 nthreads: int = 0) -> None:
    """Apply one k-qubit matrix in place (the generic set-id kernel)."""
    lib = _load()
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == (1 << n)
    k = len(qubits)
    u = np.ascontiguousarray(u, np.complex128)
    assert u.shape == (1 << k, 1 << k)
    q = (ctypes.c_int * k)(*[int(x) for x in qubits])
    rc = lib.or_apply(n, _dptr(psi.view(np.float64)), k, q, _dptr(u.view(np.float64)), nthreads)
    if rc != 0:
        raise ValueError(f"or_apply failed ({rc}) for qubits {qubits}")


def simulate(circ, params: Optional[np.ndarray] = None, psi0: Optional[np.ndarray] = None,
             nthreads: int = 0, gates: Optional[Iterable] = None) -> np.ndarray:
    """Gate-by-gate FP64 sweep.  Starts at |0...0> unless psi0 is given."""
    n = circ.n
    if psi0 is None:
        psi = np.zeros(1 << n, np.complex128)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, np.complex128, copy=True)
    for g in (circ.gates if gates is None else gates):
        apply_matrix(psi, n, g.qubits, gate_matrix(g, params), nthreads)
    return psi


def norm2(psi: np.ndarray, nthreads: int = 0) -> float:
    psi = np.ascontiguousarray(psi, np.complex128)
    n = int(psi.size).bit_length() - 1
    return float(_load().or_norm2(n, _dptr(psi.view(np.float64)), nthreads))


def pauli_term(psi: np.ndarray, x: int, z: int, nthreads: int = 0) -> complex:
    """<psi| i^{|x&z|} X^x Z^z |psi>."""
    psi = np.ascontiguousarray(psi, np.complex128)
    n = int(psi.size).bit_length() - 1
    re = ctypes.c_double()
    im = ctypes.c_double()
    _load().or_pauli_expect(n, _dptr(psi.view(np.float64)), int(x), int(z),
                            ctypes.byref(re), ctypes.byref(im), nthreads)
    ph = (1j) ** (bin(int(x) & int(z)).count("1") % 4)
    return ph * complex(re.value, im.value)


def expect(psi: np.ndarray, pauli, nthreads: int = 0) -> float:
    """sum_k c_k Re <psi|P_k|psi> (terms summed in fixed order)."""
    tot = 0.0
    for c, x, z in zip(pauli.coeff, pauli.x_mask, pauli.z_mask):
        tot += float(c) * pauli_term(psi, int(x), int(z), nthreads).real
    return tot


def inner(a: np.ndarray, b: np.ndarray, nthreads: int = 0) -> complex:
    a = np.ascontiguousarray(a, np.complex128)
    b = np.ascontiguousarray(b, np.complex128)
    n = int(a.size).bit_length() - 1
    re = ctypes.c_double()
    im = ctypes.c_double()
    _load().or_inner(n, _dptr(a.view(np.float64)), _dptr(b.view(np.float64)),
                     ctypes.byref(re), ctypes.byref(im), nthreads)
    return complex(re.value, im.value)


def energy(circ, params, pauli, psi0=None, nthreads: int = 0) -> float:
    return expect(simulate(circ, params, psi0, nthreads), pauli, nthreads)


def _param_gates(circ) -> dict:
    occ = {}
    for i, g in enumerate(circ.gates):
        if g.param >= 0:
            occ.setdefault(g.param, []).append(i)
    return occ


def grad_param_shift(circ, params: np.ndarray, pauli, psi0=None,
                     which: Optional[Sequence[int]] = None, nthreads: int = 0) -> np.ndarray:
    """dE/dtheta_p by the two-term shift rule, summed over every gate that
    uses parameter p: [E(theta + pi/2) - E(theta - pi/2)] / 2 per occurrence."""
    params = np.asarray(params, np.float64)
    occ = _param_gates(circ)
    idx = range(circ.n_params) if which is None else which
    out = np.zeros(len(list(idx)) if which is not None else circ.n_params)
    for oi, p in enumerate(idx):
        tot = 0.0
        for gi in occ.get(p, []):
            for sgn in (+1.0, -1.0):
                gl = list(circ.gates)
                g = gl[gi]
                th = float(params[p]) + sgn * np.pi / 2
                gl[gi] = type(g)(g.op, g.qubits, -1, th, g.mat)
                e = expect(simulate(circ, params, psi0, nthreads, gates=gl), pauli, nthreads)
                tot += 0.5 * sgn * e
        out[oi] = tot
    return out


def grad_fd(circ, params: np.ndarray, pauli, h: float = 1e-4, psi0=None,
            which: Optional[Sequence[int]] = None, nthreads: int = 0) -> np.ndarray:
    """Central finite differences (E(theta+h) - E(theta-h)) / 2h."""
    params = np.asarray(params, np.float64)
    idx = list(range(circ.n_params) if which is None else which)
    out = np.zeros(len(idx))
    for oi, p in enumerate(idx):
        pp = params.copy(); pp[p] += h
        pm = params.copy(); pm[p] -= h
        out[oi] = (energy(circ, pp, pauli, psi0, nthreads) -
                   energy(circ, pm, pauli, psi0, nthreads)) / (2 * h)
    return out


def apply_op_list(psi: np.ndarray, n: int, ops: List, nthreads: int = 0) -> np.ndarray:
    """Apply a list of (qubits, matrix) pairs (used to evaluate exported
    plans and other explicit operator lists)."""
    psi = np.array(psi, np.complex128, copy=True)
    for qs, u in ops:
        apply_matrix(psi, n, qs, u, nthreads)
    return psi


def sample(psi: np.ndarray, uniforms: np.ndarray) -> np.ndarray:
    """Outcomes of measuring every qubit (Sec. 2: outcome j has probability
    |alpha_j|^2; Sec. 3 notes that measurements follow from the amplitudes
    once all are known), one per random number u in [0, 1): the smallest j
    whose cumulative probability, sum_{i <= j} |alpha_i|^2, exceeds
    u * ||psi||^2.  FP64 throughout; a u whose target rounds to the total maps
    to the last outcome of nonzero probability."""
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    cdf = np.cumsum(p)
    u = np.asarray(uniforms, dtype=np.float64)
    if np.any(u < 0.0) or np.any(u >= 1.0):
        raise ValueError("uniforms must lie in [0, 1)")
    total = cdf[-1]
    if not total > 0.0:
        raise ValueError("state has zero norm")
    j = np.searchsorted(cdf, u * total, side="right")
    last = int(np.flatnonzero(p > 0.0)[-1])
    return np.minimum(j, last).astype(np.uint64)
