"""Helpers for the GPU parity tests (comparison metrics and layout changes)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_to_soa(f):
    """(nz, ny, nx, 27) oracle layout -> (27, nz, ny, nx) library layout."""
    return np.ascontiguousarray(np.moveaxis(f, -1, 0))


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def rel_vec(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / scale)
