"""Writes FP64 oracle amplitudes that the benchmark's other sweeps are
checked against:

  grid4x8_cut24_amplitudes.txt  the 24-qubit cut (qubits 0-23, gates entirely
                                inside them) of the 32-qubit 4x8 grid circuit
                                with 40 cycles, seed 1005, from |0...0>
  line12_amplitudes.txt         the 12-qubit line circuit (10 layers,
                                seed 1000), from |0...0>
  grid2x11_amplitudes.txt       the 22-qubit 2x11 grid circuit (20 cycles,
                                seed 1006), from |0...0> (the width-22
                                version of the Schroedinger-Feynman workload)

each as a seeded sample of amplitudes (the first and last 16 indices plus
2048 random ones; all 4096 for the line) and the norm.  Only the oracle
computes these values.

    python tests/golden/make_sweep_cuts.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from tests.golden.make_grid33_cut28 import sample_indices  # noqa: E402


def write(path, title, circ, idx):
    psi = oracle.simulate(circ)
    nrm = oracle.norm2(psi)
    with open(path, "w") as f:
        f.write(f"# FP64 oracle amplitudes of {title}, from |0...0>\n")
        f.write(f"# written by tests/golden/make_sweep_cuts.py; gates {len(circ)}\n")
        f.write(f"norm2 {float(nrm)!r}\n")
        for j in idx:
            f.write(f"{int(j)} {float(psi[j].real)!r} {float(psi[j].imag)!r}\n")


def main() -> None:
    c = W.grid_circuit(4, 8, 40, seed=1005).cut(24)
    write(os.path.join(HERE, "grid4x8_cut24_amplitudes.txt"),
          "the 24-qubit cut of the 4x8 grid circuit (40 cycles, seed 1005)", c, sample_indices(c.n))
    g = W.grid_circuit(2, 11, 20, seed=1006)
    write(os.path.join(HERE, "grid2x11_amplitudes.txt"), "the 2x11 grid circuit (20 cycles, seed 1006)", g,
          sample_indices(g.n))
    line = W.line_circuit(12, 10, seed=1000)
    write(os.path.join(HERE, "line12_amplitudes.txt"), "the 12-qubit line circuit (10 layers, seed 1000)",
          line, np.arange(1 << 12))


if __name__ == "__main__":
    main()
