"""Readers for the fixtures in this folder: values transcribed from the paper,
and oracle values written by the scripts here."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def matrices():
    out = {}
    name = None
    rows = []
    with open(os.path.join(HERE, "paper_matrices.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "|" in line:
                if name is not None:
                    out[name] = np.array(rows, np.complex128)
                name = line.split("|")[0].strip()
                rows = []
            else:
                rows.append([complex(x) for x in line.split()])
    if name is not None:
        out[name] = np.array(rows, np.complex128)
    return out


def bitmasks():
    out = {}
    with open(os.path.join(HERE, "paper_bitmasks.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _cite, vals = [x.strip() for x in line.split("|")]
            out[key] = vals.split()
    return out


def grid33_cut28():
    """(indices, amplitudes, norm2) written by make_grid33_cut28.py."""
    return amplitudes("grid33_cut28_amplitudes.txt")


def amplitudes(name):
    """(indices, amplitudes, norm2) of an amplitude-sample fixture."""
    idx, amp, nrm = [], [], None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "norm2":
                nrm = float(parts[1])
                continue
            idx.append(int(parts[0]))
            amp.append(complex(float(parts[1]), float(parts[2])))
    return np.array(idx, np.uint64), np.array(amp, np.complex128), nrm


def ansatz20_gradients():
    """(param indices, {set: energy}, {set: grads}) written by
    make_config_gradients.py for the 20-qubit ansatz."""
    sel, en, gr = None, {}, {}
    with open(os.path.join(HERE, "ansatz20_gradients.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "params":
                sel = np.array([int(x) for x in p[1:]], np.int64)
            elif p[0] == "set" and p[2] == "energy":
                en[int(p[1])] = float(p[3])
            elif p[0] == "set" and p[2] == "grad":
                gr[int(p[1])] = np.array([float(x) for x in p[3:]])
    return sel, en, gr


def batch_wide_gradients():
    """{item: {"n", "gates", "energy", optional "params", "grad"}} written by
    make_config_gradients.py for the widest circuits of the batch."""
    out = {}
    with open(os.path.join(HERE, "batch_wide_gradients.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            i = int(p[1])
            d = out.setdefault(i, {})
            if p[2] == "n":
                d["n"], d["gates"], d["energy"] = int(p[3]), int(p[5]), float(p[7])
            elif p[2] == "params":
                d["params"] = np.array([int(x) for x in p[3:]], np.int64)
            elif p[2] == "grad":
                d["grad"] = np.array([float(x) for x in p[3:]])
    return out
