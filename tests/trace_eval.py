"""Evaluate a planner trace (sv_plan_trace text) on a state vector in FP64.

Each line is applied from its definition in include/sv.h; dense blocks go
through the oracle's generic set-id kernel.  This checks the planner's
algebra (reordering, butterfly decomposition, lazily applied phases,
scales, gradient placement) against the gate-by-gate oracle without a GPU.
"""
import numpy as np

import oracle

W8 = np.exp(1j * np.pi / 4)


def _bits(n):
    j = np.arange(1 << n, dtype=np.int64)
    return j, [((j >> q) & 1) for q in range(n)]


def _grad_term(gen, qs, psi, lam, bit, j):
    """Im <lam|G|psi> for the generator codes of the trace."""
    if gen == 4:
        m = (bit[qs[0]] & bit[qs[1]]) == 1
        return -2.0 * float(np.imag(np.vdot(lam[m], psi[m])))
    q = qs[0]
    if gen == 1:
        gp = psi[j ^ (1 << q)]
    elif gen == 2:
        gp = np.where(bit[q] == 1, 1j, -1j) * psi[j ^ (1 << q)]
    else:
        gp = np.where(bit[q] == 1, -1.0, 1.0) * psi
    return float(np.imag(np.vdot(lam, gp)))


def _apply_line(f, line, n, psi, j, bit):
    if f[0] in ("PASS", "PHASE"):
        return
    if f[0] == "BF":
        q, m = int(f[1]), int(f[2])
        lo = j[bit[q] == 0]
        hi = lo | (1 << q)
        par = np.zeros(lo.size, np.int64)
        for p in (int(x) for x in f[3:]):
            par ^= (lo >> p) & 1
        t = (W8 ** m) * np.where(par == 1, -1.0, 1.0)
        x, y = psi[lo].copy(), psi[hi].copy()
        psi[lo] = x + t * y
        psi[hi] = x - t * y
    elif f[0] == "DENSE1":
        # DENSE1 1 q u00 u01 u10 u11 [| partners]: (x, y) <- (u00 x + s u01 y, u10 x + s u11 y)
        q = int(f[2])
        rest = f[3:]
        partners = []
        if "|" in rest:
            partners = [int(x) for x in rest[rest.index("|") + 1:]]
            rest = rest[:rest.index("|")]
        v = np.array([float(x) for x in rest])
        u = v[0::2] + 1j * v[1::2]
        lo = j[bit[q] == 0]
        hi = lo | (1 << q)
        par = np.zeros(lo.size, np.int64)
        for p in partners:
            par ^= (lo >> p) & 1
        sg = np.where(par == 1, -1.0, 1.0)
        x, y = psi[lo].copy(), psi[hi].copy()
        psi[lo] = u[0] * x + sg * u[1] * y
        psi[hi] = u[2] * x + sg * u[3] * y
    elif f[0] == "FORM":
        e = np.full(1 << n, int(f[1]), np.int64)
        for tok in f[2:]:
            key, v = tok.split(":")
            v = int(v)
            if key[0] == "a":
                e += v * bit[int(key[1:])]
            else:
                a, b = (int(x) for x in key[1:].split(","))
                e += v * bit[a] * bit[b]
        psi *= W8 ** (e % 8)
    elif f[0] in ("DENSE", "DIAG"):
        k = int(f[1])
        qs = [int(x) for x in f[2:2 + k]]
        vals = np.array([float(x) for x in f[2 + k:]])
        z = vals[0::2] + 1j * vals[1::2]
        if f[0] == "DENSE":
            oracle.apply_matrix(psi, n, qs, z.reshape(1 << k, 1 << k))
        else:
            loc = np.zeros(1 << n, np.int64)
            for t, qq in enumerate(qs):
                loc |= bit[qq] << t
            psi *= z[loc]
    elif f[0] == "PERM":
        # PERM kind q [q2]: 1 = X, 2 = Y, 3 = CNOT (control q, target q2), 4 = SWAP
        kind, q = int(f[1]), int(f[2])
        src = j.copy()
        if kind in (1, 2):
            src = j ^ (1 << q)
        elif kind == 3:
            q2 = int(f[3])
            src = np.where(bit[q] == 1, j ^ (1 << q2), j)
        else:
            q2 = int(f[3])
            src = np.where(bit[q] != bit[q2], j ^ (1 << q) ^ (1 << q2), j)
        out = psi[src]
        if kind == 2:                   # Y: (Y psi)_j = i psi_{j^q} if bit q of j is 1, else -i
            out = np.where(bit[q] == 1, 1j, -1j) * out
        psi[:] = out
    elif f[0] == "SCALE":
        psi *= float(f[1])
    else:
        raise ValueError(f"unknown trace line: {line}")


def evaluate(trace: str, n: int, psi0: np.ndarray, lam0: np.ndarray = None):
    """Apply the trace to psi0 (and to lam0 when given: adjoint plans).
    Returns the final state (or (psi, lam)) and {parameter: gradient} summed
    over the GRAD lines (0.0 entries when no lam0 is given)."""
    states = [np.array(psi0, np.complex128, copy=True)]
    if lam0 is not None:
        states.append(np.array(lam0, np.complex128, copy=True))
    j, bit = _bits(n)
    grads = {}
    for line in trace.splitlines():
        f = line.split()
        if not f:
            continue
        if f[0] == "GRAD":
            p, gen, sc = int(f[1]), int(f[2]), float(f[3])
            v = 0.0
            if lam0 is not None:
                v = sc * _grad_term(gen, [int(x) for x in f[4:]], states[0], states[1], bit, j)
            grads[p] = grads.get(p, 0.0) + v
            continue
        for psi in states:
            _apply_line(f, line, n, psi, j, bit)
    return (states[0] if lam0 is None else tuple(states)), grads


def apply_pauli_sum(psi: np.ndarray, n: int, h) -> np.ndarray:
    """H psi for H = sum_k c_k i^{|x&z|} X^x Z^z (the observable convention)."""
    j = np.arange(1 << n, dtype=np.int64)
    out = np.zeros_like(psi)
    for c, x, z in zip(h.coeff, h.x_mask, h.z_mask):
        ph = 1j ** (bin(int(x) & int(z)).count("1") % 4)
        src = j ^ int(x)
        sg = np.array([(-1.0) ** bin(int(s) & int(z)).count("1") for s in src])
        out += c * ph * sg * psi[src]
    return out
