"""Pins of the CPU oracle on adaptive octrees (leaves on several levels).

The coarse-fine reading (2:1 balanced leaves; same-level M2L between every
pair of existing cells; a leaf near a refined cell meets that cell's children
by P2P) is pinned against facts that do not come from the oracle itself:
  * exact pair cover: for sampled sinks, every other leaf cell is accounted
    for exactly once (brute-force marking over the tree);
  * two point masses across a refinement boundary: exact Newtonian values;
  * a uniform tree gives the uniform oracle's result (a separate code path);
  * Newton's third law and the symmetric potential operator (exact for
    total-order truncation at any level mix);
  * the direct sum over all leaf cells within the method's error;
  * the workload generator's trees are 2:1 balanced (checked by brute force).
"""
import numpy as np
import pytest

import oracle as O
from paper_2412_15518_amd import workloads as W
from conftest import normwise, normwise_vec


def _touching_leaf_levels_ok(lay):
    """Brute force: leaf sub-grids that touch (face, edge or corner) differ by
    at most one level."""
    L = lay.depth
    leaves = lay.leaf_nodes
    lv = lay.level[leaves].astype(np.int64)
    lo = lay.coord[leaves].astype(np.int64) << (L - lv)[:, None]
    hi = lo + (1 << (L - lv))[:, None]
    for i in range(leaves.size):
        touch = np.all((lo <= hi[i]) & (hi >= lo[i]), axis=1)
        touch[i] = False
        if np.any(np.abs(lv[touch] - lv[i]) > 1):
            return False
    return True


@pytest.mark.parametrize("kind,nsample", [("corner", 7680), ("edge", 300), ("blob", 200)])
def test_pair_cover_exact(kind, nsample):
    lay = W.small_amr(kind)["layout"]
    N = lay.n_leaf_cells
    rng = np.random.default_rng(11)
    sinks = np.arange(N) if nsample >= N else rng.choice(N, nsample, replace=False)
    if nsample >= N:
        sinks = sinks[::16]          # every 16th cell keeps the run short
    for s in sinks:
        m = O.amr_cover(lay, s)
        assert m[s] == 0, s
        assert np.all(np.delete(m, s) == 1), (s, np.unique(m, return_counts=True))


@pytest.mark.parametrize("theta", [0.34, 0.6])
def test_pair_cover_other_opening_angles(theta):
    lay = W.small_amr("edge")["layout"]
    for s in np.random.default_rng(13).choice(lay.n_leaf_cells, 60, replace=False):
        m = O.amr_cover(lay, s, theta=theta)
        assert m[s] == 0 and np.all(np.delete(m, s) == 1), (theta, s)


def test_pair_cover_workload_sample():
    d = W.adaptive_two_polytropes(with_cotangents=False)
    lay = d["layout"]
    rng = np.random.default_rng(12)
    # sinks on every leaf level
    lvl = np.repeat(lay.level[lay.leaf_nodes], 512)
    for l in np.unique(lvl):
        for s in rng.choice(np.nonzero(lvl == l)[0], 3, replace=False):
            m = O.amr_cover(lay, s)
            assert m[s] == 0 and np.all(np.delete(m, s) == 1), (l, s)


def _mass_in(lay, level, cell):
    """Leaf-cell index of the cell with global coordinates `cell` at `level`."""
    sub = tuple(c // 8 for c in cell)
    for j, nd in enumerate(lay.leaf_nodes):
        if lay.level[nd] == level and tuple(lay.coord[nd]) == sub:
            x, y, z = (c % 8 for c in cell)
            return 512 * j + (z * 8 + y) * 8 + x
    raise KeyError((level, cell))


@pytest.mark.parametrize("pair", [((1, (8, 2, 3)), (2, (15, 5, 6))), ((2, (14, 13, 1)), (1, (8, 6, 0)))])
def test_two_masses_across_the_boundary(pair):
    """A coarse and a fine leaf cell near each other (a coarse-fine P2P pair):
    each sees -G m / r and -G m r_hat / r^2 of the other, exactly."""
    d = W.small_amr("corner")
    lay = d["layout"]
    G, h = 1.5, 0.5
    lay.G, lay.h_leaf_min = G, h
    rho = np.zeros(lay.n_leaf_cells)
    (la, ca), (lb, cb) = pair
    ia, ib = _mass_in(lay, la, ca), _mass_in(lay, lb, cb)
    rho[ia], rho[ib] = 2.0, 0.7
    L = lay.depth
    ha, hb = h * 2 ** (L - la), h * 2 ** (L - lb)
    xa, xb = (np.array(ca) + 0.5) * ha, (np.array(cb) + 0.5) * hb
    ma, mb = 2.0 * ha ** 3, 0.7 * hb ** 3
    r = xa - xb
    dist = np.linalg.norm(r)
    assert dist <= 2.5 * max(ha, hb)         # a near pair at the coarse level
    phi, g = O.amr_fmm_sinks(lay, rho, [ia, ib])
    assert phi[0] == pytest.approx(-G * mb / dist, rel=1e-14)
    assert phi[1] == pytest.approx(-G * ma / dist, rel=1e-14)
    np.testing.assert_allclose(g[:, 0], -G * mb * r / dist ** 3, rtol=1e-13)
    np.testing.assert_allclose(g[:, 1], G * ma * r / dist ** 3, rtol=1e-13)


def test_uniform_tree_matches_uniform_oracle():
    lay = W.uniform_layout(2, order="random", seed=4)
    rho_d = W.random_density(32, 3)
    phi, g = O.amr_fmm_sinks(lay, lay.dense_to_layout(rho_d))
    pu, gu = O.fmm(rho_d)
    assert normwise(phi, lay.dense_to_layout(pu)) < 1e-13
    assert normwise_vec(g, lay.dense_to_layout(gu)) < 1e-13


@pytest.mark.parametrize("kind", ["corner", "edge"])
def test_newton_third_law(kind):
    d = W.small_amr(kind)
    lay, rho = d["layout"], d["rho"]
    _, hl = W.leaf_cell_centres(lay)
    phi, g = O.amr_fmm_sinks(lay, rho)
    F = (rho * hl ** 3)[None] * g
    assert np.abs(F.sum(axis=1)).max() / np.abs(F).sum() < 1e-13


def test_potential_operator_symmetric():
    d = W.small_amr("corner")
    lay = d["layout"]
    _, hl = W.leaf_cell_centres(lay)
    rng = np.random.default_rng(5)
    a, b = rng.uniform(0, 1, lay.n_leaf_cells), rng.standard_normal(lay.n_leaf_cells)
    pa, _ = O.amr_fmm_sinks(lay, a)
    pb, _ = O.amr_fmm_sinks(lay, b)
    lhs, rhs = np.sum(a * hl ** 3 * pb), np.sum(b * hl ** 3 * pa)
    assert abs(lhs - rhs) / np.abs(a * hl ** 3 * pb).sum() < 1e-12


@pytest.mark.parametrize("kind", ["corner", "edge", "blob"])
def test_direct_sum_within_method_error(kind):
    """Order 3, theta 0.4: the uniform trees give ~3e-5 (phi) and ~1e-3 (g)
    normwise; the adaptive trees must stay at that level."""
    d = W.small_amr(kind)
    lay, rho = d["layout"], d["rho"]
    rng = np.random.default_rng(6)
    sk = rng.choice(lay.n_leaf_cells, 400, replace=False)
    phi, g = O.amr_fmm_sinks(lay, rho, sk)
    pd, gd = O.amr_direct(lay, rho, sk)
    assert normwise(phi, pd) < 1e-4
    assert normwise_vec(g, gd) < 3e-3


def unbalanced_layout():
    """Root refined; of level 1 only sub-grid (0,0,0) refined; of its children
    only (1,1,1) refined: level-3 sub-grids then touch level-1 leaves."""
    nodes = [(0, (0, 0, 0), 0)]
    nodes += [(1, (b & 1, (b >> 1) & 1, b >> 2), int(b != 0)) for b in range(8)]
    nodes += [(2, (b & 1, (b >> 1) & 1, b >> 2), int(b != 7)) for b in range(8)]
    nodes += [(3, (2 + (b & 1), 2 + ((b >> 1) & 1), 2 + (b >> 2)), 1) for b in range(8)]
    level = np.array([n[0] for n in nodes], dtype=np.int32)
    coord = np.array([n[1] for n in nodes], dtype=np.int32)
    is_leaf = np.array([n[2] for n in nodes], dtype=np.uint8)
    pos = {(int(l), *map(int, c)): j for j, (l, c) in enumerate(zip(level, coord))}
    parent = np.array([-1 if l == 0 else pos[(int(l) - 1, *(int(x) >> 1 for x in c))]
                       for l, c in zip(level, coord)], dtype=np.int32)
    return W.Layout(level=level, coord=coord, parent=parent, is_leaf=is_leaf)


def test_unbalanced_tree_rejected():
    """The reading needs 2:1 balance; the oracle refuses a tree without it."""
    bad = unbalanced_layout()
    assert not _touching_leaf_levels_ok(bad)
    with pytest.raises(RuntimeError):
        O.amr_fmm_sinks(bad, np.ones(bad.n_leaf_cells))


@pytest.mark.parametrize("kind", ["corner", "edge", "blob"])
def test_small_trees_balanced(kind):
    assert _touching_leaf_levels_ok(W.small_amr(kind)["layout"])


def test_workload_tree():
    """The adaptive workload: uniform to level 3, three more levels, balanced;
    the leaf counts land in the stated range of about 600 to 2500 sub-grids."""
    d = W.adaptive_two_polytropes(with_cotangents=False)
    lay = d["layout"]
    assert lay.depth == 6
    assert np.all(lay.is_leaf[lay.level < 3] == 0)
    n_leaf = int(lay.is_leaf.sum())
    assert 600 <= n_leaf <= 2500
    assert len(np.unique(lay.level[lay.leaf_nodes])) == 4
    assert _touching_leaf_levels_ok(lay)
    assert d["rho"].shape == (lay.n_leaf_cells,) and d["rho"].min() > 0


def test_direct_sum_two_masses_on_different_levels():
    """The adaptive direct sum itself: two point masses on levels 1 and 2 give
    -G m / r and -G m r_hat / r^2 exactly, with h_l = h 2^(L - l)."""
    d = W.small_amr("corner")
    lay = d["layout"]
    G, h = 0.7, 0.25
    lay.G, lay.h_leaf_min = G, h
    rho = np.zeros(lay.n_leaf_cells)
    ia, ib = _mass_in(lay, 1, (12, 3, 9)), _mass_in(lay, 2, (2, 13, 5))
    rho[ia], rho[ib] = 1.5, 0.25
    xa, xb = (np.array([12, 3, 9]) + 0.5) * 2 * h, (np.array([2, 13, 5]) + 0.5) * h
    ma, mb = 1.5 * (2 * h) ** 3, 0.25 * h ** 3
    r = xa - xb
    dist = np.linalg.norm(r)
    phi, g = O.amr_direct(lay, rho, [ia, ib])
    assert phi[0] == pytest.approx(-G * mb / dist, rel=1e-14)
    assert phi[1] == pytest.approx(-G * ma / dist, rel=1e-14)
    np.testing.assert_allclose(g[:, 0], -G * mb * r / dist ** 3, rtol=1e-13)
    np.testing.assert_allclose(g[:, 1], G * ma * r / dist ** 3, rtol=1e-13)


def test_direct_sum_uniform_tree_matches_dense_direct_sum():
    lay = W.uniform_layout(1, order="random", seed=8)
    rho_d = W.random_density(16, 9)
    phi, g = O.amr_direct(lay, lay.dense_to_layout(rho_d))
    pd, gd = O.direct(rho_d)
    assert normwise(phi, lay.dense_to_layout(pd)) < 1e-14
    assert normwise_vec(g, lay.dense_to_layout(gd)) < 1e-14
