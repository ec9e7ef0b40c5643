"""GPU parity of the FP32 M2L (plan flag OT_FMM_M2L_FP32) against the FP64
oracle and against the library's own FP64 path, through the C ABI.

Tolerance.  The FP32 path rounds the (reduced) moments and derivative tensors
to FP32 (relative error u = 2^-24 ~ 6e-8 each) and sums the products of one
parent offset (at most 8 source children x 16 terms per output component) in
FP32 before adding them to FP64 accumulators.  A sum of n products carries at
most about n u relative to the sum of their magnitudes, so each parent
offset's contribution to a local coefficient is off by at most ~128 u ~ 1e-5
of its absolute sum.  The local expansion is dominated by a few such contributions
and everything downstream (L2L, L2P, leaf P2P) is FP64, so the normwise error
max|d phi| / max|phi| (and the same for g) is bounded by ~1e-5; measured
values are around 1e-7 and are printed.
"""
import numpy as np
import pytest

from conftest import normwise, normwise_vec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2412_15518_amd import fmm, workloads as W  # noqa: E402

TOL32 = 1e-5


def say(*a):
    print("[gpu-fp32]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmm.load_library()
    torch.cuda.set_device(0)


def to_dev(layout, dense):
    return torch.from_numpy(layout.dense_to_layout(np.ascontiguousarray(dense))).cuda()


def run(layout, rho=None, w=None, u=None, fp32=True, theta=0.4):
    plan = fmm.Plan(layout, theta=theta, m2l_fp32=fp32)
    out = {}
    if rho is not None:
        phi, g = plan.forward(to_dev(layout, rho))
        out["phi"] = layout.layout_to_dense(phi.cpu().numpy())
        out["g"] = layout.layout_to_dense(g.cpu().numpy())
    if w is not None:
        dr = plan.adjoint(to_dev(layout, w), to_dev(layout, u))
        out["drho"] = layout.layout_to_dense(dr.cpu().numpy())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("L", [1, 2, 3])
def test_forward_fp32_matches_oracle(L):
    n = 8 << L
    rho = W.random_density(n, 700 + L)
    say("forward depth", L)
    r = run(W.uniform_layout(L), rho=rho)
    po, go = O.fmm(rho)
    ep, eg = normwise(r["phi"], po), normwise_vec(r["g"], go)
    say(f"depth {L}: phi {ep:.2e}  g {eg:.2e}")
    assert ep < TOL32 and eg < TOL32


@pytest.mark.parametrize("L", [1, 2])
def test_adjoint_fp32_matches_oracle(L):
    n = 8 << L
    rng = np.random.default_rng(710 + L)
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    say("adjoint depth", L)
    r = run(W.uniform_layout(L), w=w, u=u)
    do = O.fmm_adjoint(w, u)
    e = normwise(r["drho"], do)
    say(f"depth {L}: drho {e:.2e}")
    assert e < TOL32


def test_depth0_has_no_m2l_and_matches_fp64_exactly():
    rho = W.random_density(8, 720)
    lay = W.uniform_layout(0)
    a, b = run(lay, rho=rho, fp32=True), run(lay, rho=rho, fp32=False)
    assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["g"], b["g"])


def test_fp32_against_fp64_path_full_size():
    """128^3 two-polytrope workload: forward and adjoint of the FP32 path
    against the FP64 path on the whole grid, and the forward against the
    oracle on sampled sinks."""
    cfg = W.two_polytropes()
    lay = W.uniform_layout(cfg["L"])
    say("128^3 fp32 and fp64")
    a = run(lay, rho=cfg["rho"], w=cfg["w"], u=cfg["u"], fp32=True)
    b = run(lay, rho=cfg["rho"], w=cfg["w"], u=cfg["u"], fp32=False)
    ep, eg, ed = normwise(a["phi"], b["phi"]), normwise_vec(a["g"], b["g"]), normwise(a["drho"], b["drho"])
    rel_l2 = np.linalg.norm(a["phi"] - b["phi"]) / np.linalg.norm(b["phi"])
    say(f"128^3 vs fp64 path: phi {ep:.2e} (rel L2 {rel_l2:.2e})  g {eg:.2e}  drho {ed:.2e}")
    assert ep < TOL32 and eg < TOL32 and ed < TOL32
    rng = np.random.default_rng(2025)
    n = 128
    sinks = rng.choice(n ** 3, 256, replace=False).astype(np.int64)
    po, go = O.fmm_sinks(cfg["rho"], sinks)
    assert np.abs(a["phi"].reshape(-1)[sinks] - po).max() / np.abs(b["phi"]).max() < TOL32
    gg = a["g"].reshape(3, -1)[:, sinks]
    assert np.sqrt(((gg - go) ** 2).sum(0)).max() / np.sqrt((b["g"] ** 2).sum(0)).max() < TOL32


def test_fp32_deterministic_bitwise():
    cfg = W.lognormal_sphere()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay, m2l_fp32=True)
    r = to_dev(lay, cfg["rho"])
    a = plan.forward(r)
    b = plan.forward(r)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_fp32_depth5_two_spans():
    """256^3 (depth 5): the upper M2M span also writes the FP32 moments."""
    n, L = 256, 5
    rng = np.random.default_rng(730)
    rho = rng.uniform(0.0, 1.0, (n, n, n))
    lay = W.uniform_layout(L)
    say("256^3 fp32 and fp64")
    a = run(lay, rho=rho, fp32=True)
    b = run(lay, rho=rho, fp32=False)
    ep, eg = normwise(a["phi"], b["phi"]), normwise_vec(a["g"], b["g"])
    say(f"256^3 vs fp64 path: phi {ep:.2e}  g {eg:.2e}")
    assert ep < TOL32 and eg < TOL32
