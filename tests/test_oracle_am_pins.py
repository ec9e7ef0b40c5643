"""Pins of the oracle's angular-momentum correction (spin torque per unit mass t).

The FMM with total-order truncation conserves linear momentum but not angular
momentum: the particles' total orbital torque sum_i m_i x_i x g_i is not zero.
The correction t is built so that sum_i m_i (x_i x g_i + t_i) = 0; these tests
check that against the oracle's forward g (a separate code path) for several
orders and depths, and that t is linear in rho and vanishes where the FMM is
exact."""
import numpy as np
import pytest

import oracle as O
from paper_2412_15518_amd import workloads as W


def torques(rho, p, h=1.0):
    n = rho.shape[-1]
    phi, g = O.fmm(rho, p=p, h=h)
    t = O.am_correction(rho, p=p, h=h)
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    X = np.stack([x, y, z]).reshape(3, -1).T
    m = rho.reshape(-1) * h ** 3
    orb = np.cross(X, (m[None] * g.reshape(3, -1)).T)
    spin = (m[None] * t.reshape(3, -1)).T
    return orb, spin


@pytest.mark.parametrize("L,p,kind", [(1, 2, "uniform"), (1, 3, "signed"), (1, 4, "uniform"), (2, 3, "sparse")])
def test_total_angular_momentum_conserved(L, p, kind):
    rho = W.random_density(8 << L, 10 + L + p, kind)
    orb, spin = torques(rho, p)
    scale = np.abs(orb).sum()
    assert np.abs(orb.sum(0)).max() / scale > 1e-9          # the truncation does break it
    assert np.abs(orb.sum(0) + spin.sum(0)).max() / scale < 1e-13


def test_cell_width_scaling():
    """h = 0.5: the same relation with positions, masses and kernels rescaled."""
    rho = W.random_density(16, 21)
    orb, spin = torques(rho, 3, h=0.5)
    assert np.abs(orb.sum(0) + spin.sum(0)).max() / np.abs(orb).sum() < 1e-13


def test_linear_in_rho():
    a, b = W.random_density(16, 22), W.random_density(16, 23, "signed")
    ta, tb = O.am_correction(a), O.am_correction(b)
    tc = O.am_correction(2.5 * a - 0.75 * b)
    assert np.abs(tc - (2.5 * ta - 0.75 * tb)).max() <= 1e-13 * np.abs(tc).max()


def test_single_subgrid_needs_none():
    """One sub-grid: every pair is exact (P2P or monopole M2L), t = 0."""
    t = O.am_correction(W.random_density(8, 24))
    assert not t.any()


def test_sinks_match_whole_grid():
    rho = W.random_density(16, 25)
    t = O.am_correction(rho)
    sk = np.array([0, 77, 1000, 4095])
    ts = O.am_correction(rho, sinks=sk)
    assert np.array_equal(ts, t.reshape(3, -1)[:, sk])
