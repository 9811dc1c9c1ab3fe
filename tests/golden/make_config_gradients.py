"""Writes FP64 oracle values for the gradient workloads at their own sizes:

  ansatz20_gradients.txt  20-qubit ansatz, 10 layers of RY, RZ + CZ ladder
                          (400 parameters), observable sum Z_i Z_{i+1} +
                          0.5 sum X_i; parameter sets 0-3 of the 64 drawn
                          with seed 3003; per set the energy and the
                          parameter-shift gradient of 20 sampled parameters.
  batch_wide_gradients.txt  the widest circuits of the 512-circuit batch
                          (10-22 qubits, 20-60 layers, seeds 4000 + i):
                          energies of sum Z_i for every item of 21-22 qubits
                          among the first 64, and parameter-shift gradients
                          of 6 sampled parameters for the two widest.

Only the oracle computes these values (gate by gate in FP64, two-term shift
rule); each energy at 22 qubits takes tens of seconds, too long inside a GPU
test, so they are stored.

    python tests/golden/make_config_gradients.py [ansatz|batch]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

ANSATZ_SETS = 4
ANSATZ_PARAMS = 20
BATCH_SCAN = 64
BATCH_GRAD_ITEMS = 2
BATCH_PARAMS = 6


def ansatz_param_sample(n_params: int) -> np.ndarray:
    return np.sort(np.random.default_rng(20).choice(n_params, ANSATZ_PARAMS, replace=False))


def batch_param_sample(n_params: int, item: int) -> np.ndarray:
    return np.sort(np.random.default_rng(22 + item).choice(n_params, BATCH_PARAMS, replace=False))


def write_ansatz() -> None:
    c = W.ansatz_circuit(20, 10)
    h = W.ansatz_observable(20)
    th = W.uniform_params(64, c.n_params, 3003)
    sel = ansatz_param_sample(c.n_params)
    with open(os.path.join(HERE, "ansatz20_gradients.txt"), "w") as f:
        f.write("# FP64 oracle: 20-qubit ansatz (10 layers, 400 params), theta = uniform_params(64, 400, 3003)\n")
        f.write("# observable sum Z_i Z_{i+1} + 0.5 sum X_i; two-term parameter-shift gradients\n")
        f.write("# written by tests/golden/make_config_gradients.py\n")
        f.write("params " + " ".join(str(int(p)) for p in sel) + "\n")
        for b in range(ANSATZ_SETS):
            e = oracle.energy(c, th[b], h)
            g = oracle.grad_param_shift(c, th[b], h, which=list(sel))
            f.write(f"set {b} energy {float(e)!r}\n")
            f.write(f"set {b} grad " + " ".join(repr(float(x)) for x in g) + "\n")
            f.flush()


def write_batch() -> None:
    circs = W.batch_circuits(BATCH_SCAN, 10, 22, 20, 60, seed0=4000)
    wide = [i for i, c in enumerate(circs) if c.n >= 21]
    by_size = sorted(wide, key=lambda i: -(circs[i].n * 10000 + len(circs[i])))
    grad_items = set(by_size[:BATCH_GRAD_ITEMS])
    with open(os.path.join(HERE, "batch_wide_gradients.txt"), "w") as f:
        f.write(f"# FP64 oracle: items of 21-22 qubits among the first {BATCH_SCAN} of batch_circuits(512, 10, 22, 20, 60)\n")
        f.write("# params of item i = uniform_params(1, n_params, 4000 + i)[0]; observable sum Z_i\n")
        f.write("# written by tests/golden/make_config_gradients.py\n")
        for i in wide:
            c = circs[i]
            p = W.uniform_params(1, c.n_params, 4000 + i)[0]
            h = W.z_sum(c.n)
            e = oracle.energy(c, p, h)
            f.write(f"item {i} n {c.n} gates {len(c)} energy {float(e)!r}\n")
            if i in grad_items:
                sel = batch_param_sample(c.n_params, i)
                g = oracle.grad_param_shift(c, p, h, which=list(sel))
                f.write(f"item {i} params " + " ".join(str(int(x)) for x in sel) + "\n")
                f.write(f"item {i} grad " + " ".join(repr(float(x)) for x in g) + "\n")
            f.flush()


if __name__ == "__main__":
    what = sys.argv[1:] or ["ansatz", "batch"]
    if "ansatz" in what:
        write_ansatz()
    if "batch" in what:
        write_batch()
