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
    idx, amp, nrm = [], [], None
    with open(os.path.join(HERE, "grid33_cut28_amplitudes.txt")) as f:
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
