"""Writes grid33_cut28_amplitudes.txt: FP64 oracle amplitudes of the 28-qubit
cut (qubits 0-27, gates entirely inside them) of the 33-qubit 3x11 grid
circuit with 40 cycles, seed 1002, started from |0...0>.

Only the oracle computes these values.  The 28-qubit oracle run takes
several minutes on a few cores, too long inside a GPU test, so a seeded
sample of amplitudes and the norm are stored.

    python tests/golden/make_grid33_cut28.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "grid33_cut28_amplitudes.txt")


def sample_indices(n: int, count: int = 2048, seed: int = 28) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = np.concatenate([np.arange(16), (1 << n) - 16 + np.arange(16), rng.integers(0, 1 << n, size=count)])
    return np.unique(idx.astype(np.int64))


def main() -> None:
    c = W.grid33().cut(28)
    psi = oracle.simulate(c)
    nrm = oracle.norm2(psi)
    idx = sample_indices(c.n)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle amplitudes of the 28-qubit cut of the 3x11 grid circuit\n")
        f.write("# (40 cycles, seed 1002; qubits 0-27, gates entirely inside them), from |0...0>.\n")
        f.write(f"# written by tests/golden/make_grid33_cut28.py; gates {len(c)}\n")
        f.write(f"norm2 {float(nrm)!r}\n")
        for j in idx:
            f.write(f"{int(j)} {float(psi[j].real)!r} {float(psi[j].imag)!r}\n")


if __name__ == "__main__":
    main()
