"""GPU angular-momentum correction (ot_fmm_am_correction) against the oracle.

t is linear in rho and FP64; the bar is 1e-12 normwise (per-cell Euclidean
norm).  At 128^3 the oracle is evaluated on sampled cells, and the exact
identity sum_i m_i (x_i x g_i + t_i) = 0 is checked on the whole grid with the
GPU's own forward g."""
import numpy as np
import pytest

from conftest import normwise_vec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2412_15518_amd import fmm, workloads as W  # noqa: E402

TOL = 1e-12


def say(*a):
    print("[gpu-am]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmm.load_library()
    torch.cuda.set_device(0)


def gpu_t(lay, rho, plan=None):
    plan = plan or fmm.Plan(lay, am_correction=True)
    t = plan.am_correction(torch.from_numpy(lay.dense_to_layout(np.ascontiguousarray(rho))).cuda())
    torch.cuda.synchronize()
    return lay.layout_to_dense(t.cpu().numpy())


@pytest.mark.parametrize("L,kind", [(1, "uniform"), (2, "signed")])
def test_whole_grid_matches_oracle(L, kind):
    lay = W.uniform_layout(L, order="random", seed=30 + L)
    rho = W.random_density(8 << L, 31 + L, kind)
    say("am correction, depth", L)
    t = gpu_t(lay, rho)
    to = O.am_correction(rho)
    assert normwise_vec(t.reshape(3, -1), to.reshape(3, -1)) < TOL


def test_fp32_m2l_plan_gives_the_same_t():
    """The correction reads only the FP64 upward pass: an FP32-M2L plan
    returns the same bits."""
    lay = W.uniform_layout(3)
    rho = torch.from_numpy(lay.dense_to_layout(W.random_density(64, 35))).cuda()
    t64 = fmm.Plan(lay, am_correction=True).am_correction(rho)
    t32 = fmm.Plan(lay, am_correction=True, m2l_fp32=True).am_correction(rho)
    torch.cuda.synchronize()
    assert torch.equal(t64, t32)


def test_single_subgrid_is_zero():
    lay = W.uniform_layout(0)
    t = gpu_t(lay, W.random_density(8, 33))
    assert not t.any()


def test_needs_the_flag():
    lay = W.uniform_layout(1)
    p = fmm.Plan(lay)
    with pytest.raises(fmm.OTFMMError) as e:
        p.am_correction(torch.zeros(lay.n_leaf_cells, dtype=torch.float64, device="cuda"))
    assert e.value.status == fmm.INVALID_ARGUMENT


def test_full_size_sampled_and_conservation():
    """128^3 two polytropes: sampled cells against the oracle, and the total
    angular momentum of forces plus spin torques, with the GPU forward."""
    cfg = W.two_polytropes(with_cotangents=False)
    lay = W.uniform_layout(4)
    rho = cfg["rho"]
    say("am correction 128^3")
    plan = fmm.Plan(lay, am_correction=True)
    rd = torch.from_numpy(lay.dense_to_layout(rho)).cuda()
    t = plan.am_correction(rd)
    phi, g = plan.forward(rd)
    torch.cuda.synchronize()
    t = lay.layout_to_dense(t.cpu().numpy())
    g = lay.layout_to_dense(g.cpu().numpy())
    sk = np.random.default_rng(34).choice(128 ** 3, 96, replace=False)
    to = O.am_correction(rho, sinks=sk)
    assert normwise_vec(t.reshape(3, -1)[:, sk], to) < TOL
    c = np.arange(128) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    X = np.stack([x, y, z]).reshape(3, -1).T
    m = rho.reshape(-1)
    orb = np.cross(X, (m[None] * g.reshape(3, -1)).T)
    spin = (m[None] * t.reshape(3, -1)).T
    say("orbital torque", orb.sum(0), "with the correction", orb.sum(0) + spin.sum(0))
    assert np.abs(orb.sum(0) + spin.sum(0)).max() / np.abs(orb).sum() < 1e-12


def test_depth3_sampled_and_conservation():
    """64^3, random node order: every Pi level is one whose parent offsets the
    tiled kernel splits over several workgroups (levels 0..2), each folded
    into its children's; sampled cells against the oracle, and the exact
    torque balance with the GPU forward."""
    lay = W.uniform_layout(3, order="random", seed=36)
    rho = W.random_density(64, 37, "signed")
    say("am correction, depth 3")
    plan = fmm.Plan(lay, am_correction=True)
    rd = torch.from_numpy(lay.dense_to_layout(rho)).cuda()
    t = plan.am_correction(rd)
    phi, g = plan.forward(rd)
    torch.cuda.synchronize()
    t = lay.layout_to_dense(t.cpu().numpy())
    g = lay.layout_to_dense(g.cpu().numpy())
    sk = np.random.default_rng(38).choice(64 ** 3, 256, replace=False)
    to = O.am_correction(rho, sinks=sk)
    assert normwise_vec(t.reshape(3, -1)[:, sk], to) < TOL
    c = np.arange(64) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    X = np.stack([x, y, z]).reshape(3, -1).T
    m = rho.reshape(-1)
    orb = np.cross(X, (m[None] * g.reshape(3, -1)).T)
    spin = (m[None] * t.reshape(3, -1)).T
    assert np.abs(orb.sum(0) + spin.sum(0)).max() / np.abs(orb).sum() < 1e-12
