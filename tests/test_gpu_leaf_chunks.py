"""Stencil chunks of the leaf passes (ot_fmm_plan_set_leaf_chunks, the size
rule and OT_FMM_AUTOTUNE), through the C ABI.

Every chunk count 1..8 must give the oracle's result to the FP64 bar, the
counts must agree with each other to rounding (only the order of the leaf
sums changes), and a plan must repeat its result bit for bit.
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
    print("[gpu-chunks]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmm.load_library()
    torch.cuda.set_device(0)


def to_dev(lay, a):
    return torch.from_numpy(lay.dense_to_layout(np.ascontiguousarray(a))).cuda()


@pytest.mark.parametrize("L", [1, 2, 3])
def test_every_chunk_count_matches_oracle(L):
    n = 8 << L
    rng = np.random.default_rng(800 + L)
    rho = rng.uniform(0.0, 1.0, (n, n, n))
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    lay = W.uniform_layout(L)
    plan = fmm.Plan(lay)
    inf = plan.info()
    say(f"depth {L}: size rule gives {inf['leaf_chunks_forward']} / {inf['leaf_chunks_adjoint']} chunks")
    assert 1 <= inf["leaf_chunks_forward"] <= 8 and inf["leaf_chunks_adjoint"] == inf["leaf_chunks_forward"]
    po, go = O.fmm(rho)
    do = O.fmm_adjoint(w, u)
    r, wd, ud = to_dev(lay, rho), to_dev(lay, w), to_dev(lay, u).reshape(-1)
    first = None
    for c in range(1, 9):
        plan.set_leaf_chunks(c, c)
        phi, g = plan.forward(r)
        dr = plan.adjoint(wd, ud)
        torch.cuda.synchronize()
        ph = lay.layout_to_dense(phi.cpu().numpy())
        gg = lay.layout_to_dense(g.cpu().numpy())
        dd = lay.layout_to_dense(dr.cpu().numpy())
        e = (normwise(ph, po), normwise_vec(gg, go), normwise(dd, do))
        say(f"  {c} chunks: phi {e[0]:.2e} g {e[1]:.2e} drho {e[2]:.2e}")
        assert max(e) < TOL
        if first is None:
            first = (ph, gg, dd)
        else:
            assert normwise(ph, first[0]) < 1e-14 and normwise_vec(gg, first[1]) < 1e-14
            assert normwise(dd, first[2]) < 1e-14


def test_autotuned_plan_is_valid_and_repeats():
    cfg = W.lognormal_sphere()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay, autotune=True)
    inf = plan.info()
    say("autotuned chunks (64^3):", inf["leaf_chunks_forward"], inf["leaf_chunks_adjoint"])
    assert inf["leaf_chunks_forward"] in (1, 2, 4, 8) and inf["leaf_chunks_adjoint"] in (1, 2, 4, 8)
    r = to_dev(lay, cfg["rho"])
    a = plan.forward(r)
    b = plan.forward(r)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    ref = fmm.Plan(lay)
    c = ref.forward(r)
    torch.cuda.synchronize()
    assert normwise(a[0].cpu().numpy(), c[0].cpu().numpy()) < 1e-14


def test_size_rule():
    """The size rule: the smallest power of two giving >= 16384 waves per leaf
    launch, at most 8 -- 8 chunks up to 64^3, 4 at 128^3 (4096 leaf blocks),
    1 at 256^3 (32768 blocks)."""
    for L, c in ((1, 8), (3, 8), (4, 4), (5, 1)):
        inf = fmm.Plan(W.uniform_layout(L)).info()
        assert inf["leaf_chunks_forward"] == c and inf["leaf_chunks_adjoint"] == c, (L, inf["leaf_chunks_forward"])
