"""GPU parity on adaptive octrees (leaf sub-grids on several levels), through
the C ABI, against the CPU oracle's adaptive FMM (2:1 balanced trees; same
reading of the coarse-fine pairs).

Tolerance as for uniform trees: 1e-12 normwise for the FP64 path (rounding
order only).  The adjoint is checked through the dot-product identity
sum(w phi(rho) + u . g(rho)) = sum(rho drho(w, u)) with the oracle's forward
on several densities, and at the workload size against the GPU's own
forward on the whole tree.
"""
import numpy as np
import pytest

from conftest import normwise, normwise_vec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2412_15518_amd import fmm, workloads as W  # noqa: E402

TOL = 1e-12


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmm.load_library()
    torch.cuda.set_device(0)


def forward(plan, rho):
    phi, g = plan.forward(torch.from_numpy(np.ascontiguousarray(rho)).cuda())
    torch.cuda.synchronize()
    return phi.cpu().numpy(), g.cpu().numpy()


def adjoint(plan, w, u):
    dr = plan.adjoint(torch.from_numpy(np.ascontiguousarray(w)).cuda(),
                      torch.from_numpy(np.ascontiguousarray(u)).cuda())
    torch.cuda.synchronize()
    return dr.cpu().numpy()


@pytest.mark.parametrize("kind", ["corner", "edge"])
def test_forward_whole_tree(kind):
    d = W.small_amr(kind)
    lay, rho = d["layout"], d["rho"]
    say("amr forward", kind, lay.n_nodes, "nodes")
    plan = fmm.Plan(lay)
    phi, g = forward(plan, rho)
    po, go = O.amr_fmm_sinks(lay, rho)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


@pytest.mark.parametrize("theta", [0.34, 0.6])
def test_forward_other_opening_angles(theta):
    """Near radius 2.94 and 1.67 cells: other stencils, coarse-fine reaches and
    tables, against the oracle on the whole tree."""
    d = W.small_amr("edge")
    lay, rho = d["layout"], d["rho"]
    say("amr forward theta", theta)
    phi, g = forward(fmm.Plan(lay, theta=theta), rho)
    po, go = O.amr_fmm_sinks(lay, rho, theta=theta)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


def test_forward_sampled_sinks_three_levels():
    d = W.small_amr("blob")
    lay, rho = d["layout"], d["rho"]
    say("amr forward blob")
    phi, g = forward(fmm.Plan(lay), rho)
    sk = np.random.default_rng(3).choice(lay.n_leaf_cells, 3000, replace=False)
    po, go = O.amr_fmm_sinks(lay, rho, sk)
    assert normwise(phi[sk], po) < TOL
    assert normwise_vec(g[:, sk], go) < TOL


@pytest.mark.parametrize("kind", ["corner", "edge"])
def test_adjoint_dot_product_with_oracle_forward(kind):
    d = W.small_amr(kind)
    lay = d["layout"]
    N = lay.n_leaf_cells
    rng = np.random.default_rng(21)
    w, u = rng.standard_normal(N), rng.standard_normal((3, N))
    say("amr adjoint", kind)
    dr = adjoint(fmm.Plan(lay), w, u)
    for probe in range(3):
        rho = rng.uniform(0.0, 1.0, N) if probe else d["rho"]
        po, go = O.amr_fmm_sinks(lay, rho)
        lhs = np.sum(w * po) + np.sum(u * go)
        rhs = np.sum(rho * dr)
        assert abs(lhs - rhs) / (np.abs(w * po).sum() + np.abs(u * go).sum()) < TOL, probe


def test_adjoint_potential_part_is_the_forward():
    """With u = 0 the adjoint is the potential operator, which is symmetric in
    the masses, applied to w as masses: drho = h_l^3 phi(rho = w / h_l^3)."""
    d = W.small_amr("edge")
    lay = d["layout"]
    _, hl = W.leaf_cell_centres(lay)
    w = np.random.default_rng(22).standard_normal(lay.n_leaf_cells)
    plan = fmm.Plan(lay)
    say("amr adjoint vs forward")
    dr = adjoint(plan, w, np.zeros((3, lay.n_leaf_cells)))
    pw, _ = forward(plan, w / hl ** 3)
    assert normwise(dr, hl ** 3 * pw) < TOL


def test_repeat_bitwise_and_momentum():
    d = W.small_amr("edge")
    lay, rho = d["layout"], d["rho"]
    plan = fmm.Plan(lay)
    say("amr repeat")
    p1, g1 = forward(plan, rho)
    p2, g2 = forward(plan, rho)
    assert np.array_equal(p1, p2) and np.array_equal(g1, g2)
    _, hl = W.leaf_cell_centres(lay)
    F = (rho * hl ** 3)[None] * g1
    assert np.abs(F.sum(axis=1)).max() / np.abs(F).sum() < 1e-13


def test_autotuned_and_set_chunks_agree():
    """Per-level chunk counts from the timing tuner, and counts set by hand,
    change only the rounding."""
    d = W.small_amr("blob")
    lay, rho = d["layout"], d["rho"]
    say("amr autotune")
    p0 = fmm.Plan(lay)
    p1 = fmm.Plan(lay, autotune=True)
    phi0, g0 = forward(p0, rho)
    phi1, g1 = forward(p1, rho)
    assert normwise(phi1, phi0) < 1e-14 and normwise_vec(g1, g0) < 1e-14
    for c in (1, 8):
        p0.set_leaf_chunks(c, c)
        phic, gc = forward(p0, rho)
        assert normwise(phic, phi0) < 1e-14 and normwise_vec(gc, g0) < 1e-14
        assert p0.info()["leaf_chunks_forward"] == c


def test_fp32_m2l_on_adaptive_tree():
    d = W.small_amr("edge")
    lay, rho = d["layout"], d["rho"]
    say("amr fp32 m2l")
    phi, g = forward(fmm.Plan(lay, m2l_fp32=True), rho)
    po, go = O.amr_fmm_sinks(lay, rho)
    assert normwise(phi, po) < 1e-5
    assert normwise_vec(g, go) < 1e-5


def test_workload_tree_sampled():
    """The adaptive workload (1296 leaf sub-grids on levels 3..6 of a 512^3
    box): sampled sinks on every leaf level against the oracle, and the
    adjoint against the GPU forward over the whole tree."""
    d = W.adaptive_two_polytropes()
    lay, rho = d["layout"], d["rho"]
    say("amr workload plan", lay.n_nodes, "nodes", lay.n_leaf_cells, "cells")
    plan = fmm.Plan(lay)
    phi, g = forward(plan, rho)
    lvl = np.repeat(lay.level[lay.leaf_nodes], 512)
    rng = np.random.default_rng(23)
    sk = np.concatenate([rng.choice(np.nonzero(lvl == l)[0], 64, replace=False) for l in np.unique(lvl)])
    po, go = O.amr_fmm_sinks(lay, rho, sk)
    assert normwise(phi[sk], po) < TOL
    assert normwise_vec(g[:, sk], go) < TOL
    say("amr workload adjoint")
    dr = adjoint(plan, d["w"], d["u"])
    lhs = np.sum(d["w"] * phi) + np.sum(d["u"] * g)
    assert abs(lhs - np.sum(rho * dr)) / (np.abs(d["w"] * phi).sum() + np.abs(d["u"] * g).sum()) < TOL
