"""Batches of independent octrees (ot_fmm_batch_*) and their HIP graphs,
through the C ABI.

The batch runs the same kernels as single plans, so every tree's output must
equal its own plan's single call bit for bit; one tree is also checked against
the oracle.  A captured graph is replayed several times, with other GPU work
and synchronisations between the replays, and each replay must equal the eager
result; the inputs are then changed in place and a replay must follow them.
"""
import numpy as np
import pytest

from conftest import normwise, normwise_vec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2412_15518_amd import fmm, workloads as W  # noqa: E402


def say(*a):
    print("[gpu-batch]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmm.load_library()
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def trees():
    ts = W.batch_of_octrees()
    out = []
    for t in ts:
        lay = t["layout"]
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        out.append(dict(t, lay=lay, plan=fmm.Plan(lay), rho_d=dev(t["rho"]), w_d=dev(t["w"]),
                        u_d=dev(t["u"]).reshape(-1)))
    say("trees:", [(t["n_leaf"], t["kind"]) for t in out])
    return out


def empty_like_fields(trees):
    phis = [torch.empty_like(t["rho_d"]) for t in trees]
    gs = [torch.empty(3 * t["rho_d"].numel(), dtype=torch.float64, device="cuda") for t in trees]
    drhos = [torch.empty_like(t["rho_d"]) for t in trees]
    return phis, gs, drhos


def singles(trees):
    ref = []
    for t in trees:
        phi, g = t["plan"].forward(t["rho_d"])
        dr = t["plan"].adjoint(t["w_d"], t["u_d"])
        ref.append((phi, g.reshape(-1), dr))
    torch.cuda.synchronize()
    return ref


@pytest.mark.parametrize("n_streams", [1, 4, 16])
def test_batch_equals_single_calls(trees, n_streams):
    say("batch of", len(trees), "trees on", n_streams, "streams")
    ref = singles(trees)
    b = fmm.Batch([t["plan"] for t in trees], n_streams=n_streams)
    phis, gs, drhos = empty_like_fields(trees)
    b.forward_into([t["rho_d"] for t in trees], phis, gs)
    b.adjoint_into([t["w_d"] for t in trees], [t["u_d"] for t in trees], drhos)
    torch.cuda.synchronize()
    for i, (phi, g, dr) in enumerate(ref):
        assert torch.equal(phis[i], phi) and torch.equal(gs[i], g) and torch.equal(drhos[i], dr), f"tree {i}"
    b.close()


def test_batch_tree_matches_oracle(trees):
    """The smallest tree of the batch against the adaptive oracle: the forward
    on every leaf cell, the adjoint through the dot-product identity."""
    i = min(range(len(trees)), key=lambda k: trees[k]["n_leaf"])
    t = trees[i]
    say("tree", i, "with", t["n_leaf"], "leaves vs the oracle")
    b = fmm.Batch([x["plan"] for x in trees], n_streams=4)
    phis, gs, drhos = empty_like_fields(trees)
    b.forward_into([x["rho_d"] for x in trees], phis, gs)
    b.adjoint_into([x["w_d"] for x in trees], [x["u_d"] for x in trees], drhos)
    torch.cuda.synchronize()
    phi = phis[i].cpu().numpy()
    g = gs[i].cpu().numpy().reshape(3, -1)
    dr = drhos[i].cpu().numpy()
    po, go = O.amr_fmm_sinks(t["lay"], t["rho"])
    e = (normwise(phi, po), normwise_vec(g, go))
    lhs = np.sum(t["w"] * po) + np.sum(t["u"] * go)
    ed = abs(lhs - np.sum(t["rho"] * dr)) / (np.abs(t["w"] * po).sum() + np.abs(t["u"] * go).sum())
    say(f"phi {e[0]:.2e} g {e[1]:.2e} adjoint identity {ed:.2e}")
    assert max(e) < 1e-12 and ed < 1e-12
    b.close()


def test_graph_replays_match_eager(trees):
    say("graph capture of the batch forward and adjoint")
    ref = singles(trees)
    b = fmm.Batch([t["plan"] for t in trees], n_streams=4)
    phis, gs, drhos = empty_like_fields(trees)
    rhos = [t["rho_d"].clone() for t in trees]
    ws = [t["w_d"].clone() for t in trees]
    us = [t["u_d"].clone() for t in trees]
    gf = b.capture_forward(rhos, phis, gs)
    ga = b.capture_adjoint(ws, us, drhos)
    for rep in range(3):
        for x in phis + gs + drhos:
            x.fill_(float("nan"))
        gf.launch()
        ga.launch()
        torch.cuda.synchronize()
        for i, (phi, g, dr) in enumerate(ref):
            assert torch.equal(phis[i], phi) and torch.equal(gs[i], g) and torch.equal(drhos[i], dr), (rep, i)
        # eager work of the program between replays
        trees[0]["plan"].forward(trees[0]["rho_d"])
        torch.cuda.synchronize()
    # the graph reads its buffers at replay time: scale the inputs
    for x in rhos + ws + us:
        x.mul_(2.0)
    gf.launch()
    ga.launch()
    torch.cuda.synchronize()
    for i, (phi, g, dr) in enumerate(ref):
        assert torch.allclose(phis[i], 2 * phi, rtol=1e-13, atol=0) and torch.allclose(drhos[i], 2 * dr, rtol=1e-13, atol=0)
    gf.close()
    ga.close()
    b.close()


def test_capture_refused_while_timing(trees):
    b = fmm.Batch([t["plan"] for t in trees[:2]], n_streams=2)
    phis, gs, _ = empty_like_fields(trees[:2])
    trees[0]["plan"].timing_begin(1)
    try:
        with pytest.raises(fmm.OTFMMError) as ei:
            b.capture_forward([t["rho_d"] for t in trees[:2]], phis, gs)
        assert ei.value.status == fmm.INVALID_ARGUMENT
    finally:
        trees[0]["plan"].timing_end()
        b.close()


def test_batch_mixed_depths_and_precisions():
    """Depths 0, 1 and 5 (no M2L, one level, two M2M spans), one FP32-M2L plan
    and one adaptive tree in one batch: every plan still gives its single
    call's bits."""
    rng = np.random.default_rng(900)
    specs = [(0, False), (1, False), (5, False), (2, True), (3, False)]
    plans, rhos, ws, us = [], [], [], []
    for L, f32 in specs:
        n = 8 << L
        lay = W.uniform_layout(L)
        plans.append(fmm.Plan(lay, m2l_fp32=f32))
        dev = lambda a, lay=lay: torch.from_numpy(lay.dense_to_layout(np.ascontiguousarray(a))).cuda()  # noqa: E731
        rhos.append(dev(rng.uniform(0.0, 1.0, (n, n, n))))
        ws.append(dev(rng.standard_normal((n, n, n))))
        us.append(dev(rng.standard_normal((3, n, n, n))).reshape(-1))
    amr = W.small_amr("edge")
    plans.append(fmm.Plan(amr["layout"]))
    na = amr["layout"].n_leaf_cells
    rhos.append(torch.from_numpy(amr["rho"]).cuda())
    ws.append(torch.from_numpy(rng.standard_normal(na)).cuda())
    us.append(torch.from_numpy(rng.standard_normal(3 * na)).cuda())
    specs = specs + [("adaptive", False)]
    say("mixed batch:", specs)
    ref = []
    for p, r, w, u in zip(plans, rhos, ws, us):
        phi, g = p.forward(r)
        ref.append((phi, g.reshape(-1), p.adjoint(w, u)))
    torch.cuda.synchronize()
    b = fmm.Batch(plans, n_streams=3)
    phis = [torch.empty_like(r) for r in rhos]
    gs = [torch.empty(3 * r.numel(), dtype=torch.float64, device="cuda") for r in rhos]
    drhos = [torch.empty_like(r) for r in rhos]
    b.forward_into(rhos, phis, gs)
    b.adjoint_into(ws, us, drhos)
    torch.cuda.synchronize()
    for i, (phi, g, dr) in enumerate(ref):
        assert torch.equal(phis[i], phi) and torch.equal(gs[i], g) and torch.equal(drhos[i], dr), specs[i]
    gf = b.capture_forward(rhos, phis, gs)
    for x in phis + gs:
        x.fill_(float("nan"))
    gf.launch()
    torch.cuda.synchronize()
    for i, (phi, g, _) in enumerate(ref):
        assert torch.equal(phis[i], phi) and torch.equal(gs[i], g), specs[i]
    gf.close()
    b.close()
