import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long statistical run")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def per_atom_ok(f, fo, fs, tol):
    """|f_i - fo_i| <= tol * fs_i for every atom (fs: the oracle's per-atom
    force scale, the sum of the magnitudes of the atom's force terms);
    returns (ok, worst ratio |df_i| / fs_i, its atom)."""
    d = np.linalg.norm(np.asarray(f, float) - np.asarray(fo, float), axis=1)
    ratio = d / np.maximum(np.asarray(fs, float), 1e-300)
    i = int(np.argmax(ratio)) if ratio.size else 0
    return bool((ratio <= tol).all()), float(ratio.max(initial=0.0)), i
