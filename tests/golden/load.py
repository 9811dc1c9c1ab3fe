"""Readers for the transcribed paper fixtures in this folder."""
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
