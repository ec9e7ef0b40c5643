"""Test configuration: the `gpu` marker and shared helpers.

Tests marked `gpu` need an MI355X (gfx950) and the built HIP library; the
rest run on any CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")


def normwise(a, b):
    """max |a - b| / max |b| (scalar fields)."""
    import numpy as np
    return float(np.abs(a - b).max() / np.abs(b).max())


def normwise_vec(a, b):
    """max_i |a_i - b_i|_2 / max_i |b_i|_2 for vector fields with the
    components on axis 0."""
    import numpy as np
    d = np.sqrt(((a - b) ** 2).sum(axis=0)).max()
    return float(d / np.sqrt((b ** 2).sum(axis=0)).max())
