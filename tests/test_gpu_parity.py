"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Tolerance: the FP64 path must match the oracle FMM (same theta, order and
tree) to 1e-12 normwise, i.e. max|d phi| / max|phi| and the same for g with
the per-cell Euclidean norm (rounding-order differences only: ~650 terms per
cell at 1.1e-16 each).  At the 128^3 size the oracle is evaluated per sink on
a sample of cells; properties that hold at any size (momentum conservation,
the adjoint identities) are checked on the whole grid.
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


def to_dev(layout, dense):
    return torch.from_numpy(layout.dense_to_layout(np.ascontiguousarray(dense))).cuda()


def gpu_forward(layout, rho, theta=0.4, plan=None):
    plan = plan or fmm.Plan(layout, theta=theta)
    say("forward", layout.depth, "theta", theta)
    phi, g = plan.forward(to_dev(layout, rho))
    torch.cuda.synchronize()
    return layout.layout_to_dense(phi.cpu().numpy()), layout.layout_to_dense(g.cpu().numpy())


def gpu_adjoint(layout, w, u, theta=0.4, plan=None):
    plan = plan or fmm.Plan(layout, theta=theta)
    say("adjoint", layout.depth, "theta", theta)
    dr = plan.adjoint(to_dev(layout, w), to_dev(layout, u))
    torch.cuda.synchronize()
    return layout.layout_to_dense(dr.cpu().numpy())


# ------------------------------------------------------------------ forward
@pytest.mark.parametrize("kind,seed", [("uniform", 1), ("signed", 2), ("sparse", 3)])
def test_single_subgrid_equals_direct_sum(kind, seed):
    lay = W.uniform_layout(0)
    rho = W.random_density(8, seed, kind)
    phi, g = gpu_forward(lay, rho)
    pd, gd = O.direct(rho)
    assert normwise(phi, pd) < TOL
    assert normwise_vec(g, gd) < TOL


@pytest.mark.parametrize("L,order,seed", [(1, "lex", 11), (1, "random", 12), (2, "morton", 13), (2, "random", 14)])
def test_forward_matches_oracle_small(L, order, seed):
    lay = W.uniform_layout(L, order=order, seed=seed)
    n = 8 << L
    rho = W.random_density(n, seed, "uniform")
    phi, g = gpu_forward(lay, rho)
    po, go = O.fmm(rho)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


@pytest.mark.parametrize("theta", [0.34, 0.5, 0.7, 1.0])
def test_forward_other_theta(theta):
    lay = W.uniform_layout(2)
    rho = W.random_density(32, 21, "signed")
    phi, g = gpu_forward(lay, rho, theta=theta)
    po, go = O.fmm(rho, theta=theta)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


def test_forward_scaled_units():
    lay = W.uniform_layout(2)
    lay.h_leaf_min = 0.37
    lay.G = 2.5
    rho = W.random_density(32, 22, "uniform")
    phi, g = gpu_forward(lay, rho)
    po, go = O.fmm(rho, h=0.37, G=2.5)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


def test_sphere_32():
    """32^3 uniform sphere: GPU == oracle FMM; accuracy against the direct sum
    is the method's (stated, ~1e-4 in phi, ~3e-3 in g)."""
    cfg = W.sphere_32()
    lay = W.uniform_layout(cfg["L"])
    phi, g = gpu_forward(lay, cfg["rho"])
    po, go = O.fmm(cfg["rho"])
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL
    pd, gd = O.direct(cfg["rho"])
    ep, eg = normwise(phi, pd), normwise_vec(g, gd)
    say(f"32^3 sphere vs direct sum: phi {ep:.3e}  g {eg:.3e}")
    assert ep < 2e-4 and eg < 5e-3


def test_lognormal_sphere_forward():
    cfg = W.lognormal_sphere()
    lay = W.uniform_layout(cfg["L"], order="morton")
    phi, g = gpu_forward(lay, cfg["rho"])
    po, go = O.fmm(cfg["rho"])
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


def test_edge_cases_zero_and_point():
    lay = W.uniform_layout(2)
    phi, g = gpu_forward(lay, np.zeros((32, 32, 32)))
    assert not phi.any() and not g.any()
    rho = np.zeros((32, 32, 32))
    rho[0, 0, 0] = 1.0          # corner cell
    rho[31, 17, 5] = -2.0
    phi, g = gpu_forward(lay, rho)
    po, go = O.fmm(rho)
    assert normwise(phi, po) < TOL
    assert normwise_vec(g, go) < TOL


def test_two_polytropes_sampled_full_size():
    """128^3 two-polytrope workload, one forward as the benchmark runs it;
    oracle evaluated per sink on 512 sampled cells (plus the domain corners)."""
    cfg = W.two_polytropes(with_cotangents=False)
    lay = W.uniform_layout(cfg["L"])
    phi, g = gpu_forward(lay, cfg["rho"])
    rng = np.random.default_rng(2024)
    n = 128
    sinks = np.concatenate([rng.choice(n ** 3, 512, replace=False),
                            [0, n - 1, n * n - 1, n ** 3 - 1, (64 * n + 64) * n + 39]]).astype(np.int64)
    say("oracle sinks", sinks.size)
    po, go = O.fmm_sinks(cfg["rho"], sinks)
    ph = phi.reshape(-1)[sinks]
    gg = g.reshape(3, -1)[:, sinks]
    assert np.abs(ph - po).max() / np.abs(phi).max() < TOL
    assert np.sqrt(((gg - go) ** 2).sum(0)).max() / np.sqrt((g ** 2).sum(0)).max() < TOL
    # whole-grid property: Newton's third law
    F = (cfg["rho"][None] * g).reshape(3, -1).sum(1)
    assert np.abs(F).max() / np.abs(cfg["rho"][None] * g).sum() < 1e-12


def test_depth5_two_tree_spans():
    """256^3 (depth 5): the M2M and L2L passes run as two spans of levels,
    the lower span taking its roots' parent expansions from memory.  Forward
    on sampled sinks and the adjoint on one z-layer against the oracle, the
    dot-product identity on the whole grid."""
    n, L = 256, 5
    rng = np.random.default_rng(505)
    rho = rng.uniform(0.0, 1.0, (n, n, n))
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    lay = W.uniform_layout(L)
    plan = fmm.Plan(lay)
    assert plan.info()["depth"] == L
    say("256^3 forward + adjoint")
    rd, wd, ud = to_dev(lay, rho), to_dev(lay, w), to_dev(lay, u)
    phi_d, g_d = plan.forward(rd)
    dr_d = plan.adjoint(wd, ud)
    torch.cuda.synchronize()
    lhs = float((wd * phi_d).sum() + (ud.reshape(3, -1) * g_d).sum())
    rhs = float((dr_d * rd).sum())
    scale = float((wd * phi_d).abs().sum() + (ud.reshape(3, -1) * g_d).abs().sum())
    assert abs(lhs - rhs) / scale < 1e-12
    phi = lay.layout_to_dense(phi_d.cpu().numpy())
    g = lay.layout_to_dense(g_d.cpu().numpy())
    dr = lay.layout_to_dense(dr_d.cpu().numpy())
    del rd, wd, ud, phi_d, g_d, dr_d
    sinks = np.concatenate([rng.choice(n ** 3, 256, replace=False),
                            [0, n - 1, n ** 3 - 1, (128 * n + 127) * n + 128]]).astype(np.int64)
    say("oracle sinks", sinks.size)
    po, go = O.fmm_sinks(rho, sinks)
    assert np.abs(phi.reshape(-1)[sinks] - po).max() / np.abs(phi).max() < TOL
    gg = g.reshape(3, -1)[:, sinks]
    assert np.sqrt(((gg - go) ** 2).sum(0)).max() / np.sqrt((g ** 2).sum(0)).max() < TOL
    z = 131
    say("oracle adjoint, z-layer", z)
    do = O.fmm_adjoint(w, u, zslab=(z, z + 1))
    assert np.abs(dr[z] - do[z]).max() / np.abs(do[z]).max() < TOL


def test_depth6_largest_supported_tree():
    """512^3 (depth 6, 134M cells), the deepest tree a plan accepts: the
    forward on sampled sinks against the oracle, and the adjoint through the
    dot-product identity on the whole grid."""
    n, L = 512, 6
    rng = np.random.default_rng(606)
    lay = W.uniform_layout(L)
    plan = fmm.Plan(lay)
    inf = plan.info()
    say(f"512^3 plan: {inf['device_bytes'] / 2**30:.1f} GiB of device memory")
    assert inf["depth"] == L
    rho = rng.uniform(0.0, 1.0, (n, n, n))
    rd = to_dev(lay, rho)
    phi_d, g_d = plan.forward(rd)
    wd = torch.randn(n ** 3, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(61))
    ud = torch.randn(3 * n ** 3, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(62))
    dr_d = plan.adjoint(wd, ud)
    torch.cuda.synchronize()
    lhs = float((wd * phi_d).sum() + (ud.reshape(3, -1) * g_d).sum())
    rhs = float((dr_d * rd).sum())
    scale = float((wd * phi_d).abs().sum() + (ud.reshape(3, -1) * g_d).abs().sum())
    say(f"dot-product identity: {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) / scale < 1e-12
    del wd, ud, dr_d, rd
    phi = lay.layout_to_dense(phi_d.cpu().numpy())
    g = lay.layout_to_dense(g_d.cpu().numpy())
    del phi_d, g_d
    sinks = np.concatenate([rng.choice(n ** 3, 64, replace=False),
                            [0, n - 1, n ** 3 - 1, (256 * n + 255) * n + 256]]).astype(np.int64)
    say("oracle sinks", sinks.size)
    po, go = O.fmm_sinks(rho, sinks)
    e_phi = np.abs(phi.reshape(-1)[sinks] - po).max() / np.abs(phi).max()
    gg = g.reshape(3, -1)[:, sinks]
    e_g = np.sqrt(((gg - go) ** 2).sum(0)).max() / np.sqrt((g ** 2).sum(0)).max()
    say(f"sinks: phi {e_phi:.2e} g {e_g:.2e}")
    assert e_phi < TOL and e_g < TOL


def test_deterministic_bitwise():
    cfg = W.lognormal_sphere()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay)
    r = to_dev(lay, cfg["rho"])
    a = plan.forward(r)
    b = plan.forward(r)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    w, u = to_dev(lay, cfg["w"]), to_dev(lay, cfg["u"])
    assert torch.equal(plan.adjoint(w, u), plan.adjoint(w, u))


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("L", [0, 1, 2])
def test_adjoint_matches_oracle_small(L):
    n = 8 << L
    rng = np.random.default_rng(300 + L)
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    lay = W.uniform_layout(L, order="random", seed=L)
    dr = gpu_adjoint(lay, w, u)
    do = O.fmm_adjoint(w, u)
    assert normwise(dr, do) < TOL


@pytest.mark.parametrize("order", ["random", "morton"])
def test_adjoint_other_layout_orders(order):
    """The adjoint reads and writes the caller's sub-grid order through the
    same leaf table as the forward."""
    n = 32
    rng = np.random.default_rng(330)
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    lay = W.uniform_layout(2, order=order, seed=7)
    dr = gpu_adjoint(lay, w, u)
    assert normwise(dr, O.fmm_adjoint(w, u)) < TOL


def test_adjoint_lognormal_sphere_matches_oracle_and_fd():
    """64^3 lognormal sphere: GPU adjoint == oracle adjoint, and central finite
    differences of L = sum w phi + sum u g through the GPU forward on the 64
    seeded cells.  F is linear, so the difference quotient has no truncation
    error; what remains is the rounding of L itself.  Each cell value is a sum
    of ~650 terms, so its rounding is ~sqrt(650) eps |value| (random walk), and
    the FD error is about sqrt(2) * 25 eps ||(w phi, u g)||_2 / (2 eps_fd)
    ~ 18 eps S2 / eps_fd.  The bar is 50 eps S2 / eps_fd (for eps_fd = 1e-6
    that is ~2e-4 of max|drho|; measured 3.3e-5)."""
    cfg = W.lognormal_sphere()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay)
    dr = gpu_adjoint(lay, cfg["w"], cfg["u"], plan=plan)
    do = O.fmm_adjoint(cfg["w"], cfg["u"])
    assert normwise(dr, do) < TOL
    rho = to_dev(lay, cfg["rho"])
    w = to_dev(lay, cfg["w"])
    u = to_dev(lay, cfg["u"]).reshape(3, -1)
    ph0, g0 = plan.forward(rho)
    S2 = float(torch.sqrt(((w * ph0) ** 2).sum() + ((u * g0) ** 2).sum()))
    machine_eps = float(np.finfo(np.float64).eps)
    pos = np.argsort(lay._leaf_index())          # dense index -> layout position
    for eps in (1e-6, 1.0):
        fd, ad = [], []
        say("finite differences", len(cfg["cells"]), "eps", eps)
        for j in cfg["cells"]:
            k = int(pos[j])
            vals = []
            for sgn in (1.0, -1.0):
                r = rho.clone()
                r[k] += sgn * eps
                ph, g = plan.forward(r)
                vals.append(float((w * ph).sum() + (u * g).sum()))
            fd.append((vals[0] - vals[1]) / (2 * eps))
            ad.append(dr.reshape(-1)[j])
        fd, ad = np.array(fd), np.array(ad)
        err = np.abs(fd - ad).max()
        bound = 50.0 * machine_eps * S2 / eps
        say(f"FD vs adjoint (eps={eps:g}, 64 cells): {err / np.abs(ad).max():.3e} relative, "
            f"bound {bound / np.abs(ad).max():.3e}")
        assert err <= bound


def test_adjoint_identities_full_size():
    """128^3: dot-product identity and, for u = 0, the adjoint equals the
    forward potential of w (the potential operator is symmetric)."""
    cfg = W.two_polytropes()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay)
    rho, w, u = to_dev(lay, cfg["rho"]), to_dev(lay, cfg["w"]), to_dev(lay, cfg["u"])
    say("128^3 forward + adjoint")
    phi, g = plan.forward(rho)
    dr = plan.adjoint(w, u)
    lhs = float((w * phi).sum() + (u.reshape(3, -1) * g).sum())
    rhs = float((dr * rho).sum())
    scale = float((w * phi).abs().sum() + (u.reshape(3, -1) * g).abs().sum())
    assert abs(lhs - rhs) / scale < 1e-12
    d0 = plan.adjoint(w, torch.zeros_like(u))
    pw, _ = plan.forward(w)
    assert float((d0 - pw).abs().max() / pw.abs().max()) < TOL


def test_autograd_function():
    lay = W.uniform_layout(1)
    plan = fmm.Plan(lay)
    rng = np.random.default_rng(5)
    rho = to_dev(lay, rng.uniform(size=(16, 16, 16))).requires_grad_(True)
    w = to_dev(lay, rng.standard_normal((16, 16, 16)))
    u = to_dev(lay, rng.standard_normal((3, 16, 16, 16))).reshape(3, -1)
    phi, g = fmm.otfmm(rho, plan)
    loss = (w * phi).sum() + (u * g).sum()
    (grad,) = torch.autograd.grad(loss, rho)
    ref = plan.adjoint(w, u)
    assert torch.allclose(grad, ref, rtol=0, atol=0)


def test_timing_api():
    lay = W.uniform_layout(2)
    plan = fmm.Plan(lay)
    r = to_dev(lay, W.random_density(32, 3))
    plan.timing_begin(4)
    for _ in range(3):
        plan.forward(r)
    plan.adjoint(r, torch.zeros((3, r.numel()), dtype=torch.float64, device=r.device))
    t = plan.timing_end()
    assert t["calls"] == 4
    assert t["phases"]["m2l"]["events"] == 4 and t["phases"]["m2l"]["ms"] > 0
    assert t["phases"]["leaf"]["events"] == 3 and t["phases"]["leaf_adj"]["events"] == 1
    assert t["phases"]["total"]["events"] == 4
    # events restricted to one phase
    plan.timing_begin(4)
    plan.timing_phases(["m2l"])
    plan.forward(r)
    plan.forward(r)
    t = plan.timing_end()
    assert t["calls"] == 2 and t["phases"]["m2l"]["events"] == 2 and t["phases"]["m2l"]["ms"] > 0
    assert all(v["events"] == 0 for k, v in t["phases"].items() if k != "m2l")
    with pytest.raises(fmm.OTFMMError):
        plan.timing_phases(["m2l"])                 # no active timing_begin
    plan.timing_begin(1)
    with pytest.raises(fmm.OTFMMError):
        fmm._check(fmm.load_library().ot_fmm_timing_phases(plan._handle, 0))
    plan.timing_end()


def test_bad_tensor_arguments_raise():
    lay = W.uniform_layout(1)
    plan = fmm.Plan(lay)
    with pytest.raises(TypeError):
        plan.forward(torch.zeros(16 ** 3, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(100, dtype=torch.float64, device="cuda"))
