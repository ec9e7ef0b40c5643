"""Pins of the CPU oracle against facts fixed by mathematics, not by itself.

Each test targets a class of plausible mistakes in the oracle:
  * 8^3 single sub-grid: FMM == direct sum exactly (every pair is exact).
  * uniform sphere: potential and field against the closed form.
  * Newton's third law, linearity and the symmetric potential operator
    (exact for total-order truncation, any p).
  * the 48 signed axis permutations of the cube (index/sign errors in the
    order-2/3 tensors and in the parity-aware stencil).
  * pair cover: every ordered leaf pair is counted exactly once.
  * convergence in p and theta towards the direct sum (dropped terms or a
    double count leave a floor).
  * derivatives of 1/r: harmonicity, homogeneity, parity, finite differences,
    and the textbook low-order forms.
  * moments after M2M equal the moment definition summed over the leaves.
  * adjoint: dot-product identity, symmetric-operator identity and finite
    differences.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_2412_15518_amd import workloads as W
from conftest import normwise, normwise_vec


# ---------------------------------------------------------------- direct sum
def test_direct_two_body_closed_form():
    """Two point masses: phi = -G m/r and g = -G m r_hat / r^2 exactly."""
    n, h, G = 8, 0.5, 2.0
    rho = np.zeros((n, n, n))
    rho[1, 2, 3] = 3.0          # [z, y, x]
    rho[6, 5, 0] = 0.5
    phi, g = O.direct(rho, h=h, G=G)
    xa = (np.array([3, 2, 1]) + 0.5) * h
    xb = (np.array([0, 5, 6]) + 0.5) * h
    ma, mb = 3.0 * h ** 3, 0.5 * h ** 3
    r = xa - xb
    d = np.linalg.norm(r)
    assert phi[1, 2, 3] == pytest.approx(-G * mb / d, rel=1e-14)
    assert phi[6, 5, 0] == pytest.approx(-G * ma / d, rel=1e-14)
    np.testing.assert_allclose(g[:, 1, 2, 3], -G * mb * r / d ** 3, rtol=1e-14)
    np.testing.assert_allclose(g[:, 6, 5, 0], G * ma * r / d ** 3, rtol=1e-14)
    # a third empty cell feels both
    xc = (np.array([0, 0, 0]) + 0.5) * h
    want = -G * (ma / np.linalg.norm(xc - xa) + mb / np.linalg.norm(xc - xb))
    assert phi[0, 0, 0] == pytest.approx(want, rel=1e-14)


def _sphere_closed_form(n, R, centre):
    """phi, g of a homogeneous sphere of mass M = sum(m), radius R (G = 1)."""
    c = np.arange(n) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    X = np.stack([x - centre[0], y - centre[1], z - centre[2]])
    r = np.sqrt((X ** 2).sum(0))
    return r, X


@pytest.mark.parametrize("which", ["direct", "fmm"])
def test_uniform_sphere_closed_form(which):
    """phi = -(GM/2R)(3 - r^2/R^2) inside, -GM/r outside; g = -GM r/R^3 inside,
    -GM r_hat/r^2 outside, with M the lattice mass and R = (3M/4pi)^(1/3).
    Cells within 2h of the surface are excluded (staircase); the remaining
    difference is the discretisation of the lattice, stated below."""
    cfg = W.sphere_32()
    rho = cfg["rho"]
    phi, g = O.direct(rho) if which == "direct" else O.fmm(rho)
    M = rho.sum()
    R = (3 * M / (4 * math.pi)) ** (1 / 3)
    r, X = _sphere_closed_form(32, R, (16.0, 16.0, 16.0))
    inside = r < R
    phi_ex = np.where(inside, -(M / (2 * R)) * (3 - r ** 2 / R ** 2), -M / np.maximum(r, 1e-300))
    gmag = np.where(inside, -M * r / R ** 3, -M / np.maximum(r, 1e-300) ** 2)
    g_ex = gmag * X / np.maximum(r, 1e-300)
    keep = np.abs(r - R) > 2.0
    ephi = np.abs(phi - phi_ex)[keep].max() / np.abs(phi_ex[keep]).max()
    eg = np.sqrt(((g - g_ex) ** 2).sum(0))[keep].max() / np.sqrt((g_ex ** 2).sum(0))[keep].max()
    # measured: phi 3.9e-3 (direct) / 3.9e-3 (fmm); g 1.6e-2 / 1.6e-2
    assert ephi < 1e-2
    assert eg < 3e-2


# ---------------------------------------------------------------- P1 exactness
@pytest.mark.parametrize("seed,kind,theta", [(1, "uniform", 0.4), (2, "signed", 0.4),
                                             (3, "sparse", 0.5), (4, "signed", 0.7)])
def test_single_subgrid_equals_direct(seed, kind, theta):
    rho = W.random_density(8, seed, kind)
    pd, gd = O.direct(rho)
    pf, gf = O.fmm(rho, theta=theta)
    assert normwise(pf, pd) < 1e-13
    assert normwise_vec(gf, gd) < 1e-13


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("p", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("theta", [0.4, 0.6])
def test_newton_third_law(p, theta):
    """sum_i m_i g_i = 0 for the FMM (total-order truncation keeps each
    far-field pair force antisymmetric)."""
    rho = W.random_density(16, 10 + p, "uniform") + 0.1
    _, g = O.fmm(rho, p=p, theta=theta)
    F = (rho[None] * g).reshape(3, -1).sum(1)
    assert np.abs(F).max() / np.abs(rho[None] * g).sum() < 1e-13


def test_linearity():
    a = W.random_density(16, 21, "signed")
    b = W.random_density(16, 22, "uniform")
    pa, ga = O.fmm(a)
    pb, gb = O.fmm(b)
    pc, gc = O.fmm(2.5 * a - 0.75 * b)
    assert normwise(pc, 2.5 * pa - 0.75 * pb) < 1e-13
    assert normwise_vec(gc, 2.5 * ga - 0.75 * gb) < 1e-13


@pytest.mark.parametrize("p", [1, 3, 4])
def test_potential_operator_symmetric(p):
    a = W.random_density(16, 31, "signed")
    b = W.random_density(16, 32, "signed")
    pa, _ = O.fmm(a, p=p)
    pb, _ = O.fmm(b, p=p)
    lhs, rhs = (a * pb).sum(), (b * pa).sum()
    assert abs(lhs - rhs) / np.abs(a * pb).sum() < 1e-12


def _signed_perms():
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product([False, True], repeat=3):
            yield perm, flips


def _apply_scalar(a, perm, flips):
    """Field b(x) = a(T^-1 x) for T = reflect-then-permute axes (x,y,z)."""
    # array axes are (z, y, x): spatial axis k lives on array axis 2 - k
    out = a
    for k in range(3):
        if flips[k]:
            out = np.flip(out, axis=2 - k)
    # permute: new spatial axis perm[k] takes old axis k
    src_axes = [None] * 3
    for k in range(3):
        src_axes[2 - perm[k]] = 2 - k
    return np.ascontiguousarray(np.transpose(out, src_axes))


def _apply_vector(g, perm, flips):
    comps = [_apply_scalar(g[k], perm, flips) * (-1.0 if flips[k] else 1.0) for k in range(3)]
    out = np.empty_like(g)
    for k in range(3):
        out[perm[k]] = comps[k]
    return out


def test_cube_symmetry_48():
    rho = W.random_density(16, 41, "uniform") * np.linspace(0.2, 1.8, 16)[None, None, :]
    phi, g = O.fmm(rho)
    for perm, flips in _signed_perms():
        rt = _apply_scalar(rho, perm, flips)
        pt, gt = O.fmm(rt)
        assert normwise(pt, _apply_scalar(phi, perm, flips)) < 1e-13, (perm, flips)
        assert normwise_vec(gt, _apply_vector(g, perm, flips)) < 1e-13, (perm, flips)


def test_cube_symmetry_32_samples():
    rho = W.random_density(32, 42, "sparse")
    phi, g = O.fmm(rho)
    for perm, flips in [((1, 2, 0), (True, False, False)), ((2, 1, 0), (False, True, True))]:
        pt, gt = O.fmm(_apply_scalar(rho, perm, flips))
        assert normwise(pt, _apply_scalar(phi, perm, flips)) < 1e-13
        assert normwise_vec(gt, _apply_vector(g, perm, flips)) < 1e-13


# ---------------------------------------------------------------- pair cover
@pytest.mark.parametrize("L,theta", [(0, 0.4), (1, 0.4), (2, 0.4), (3, 0.4), (2, 0.5), (2, 0.9), (2, 0.34)])
def test_pair_cover(L, theta):
    """Every ordered pair of distinct leaf cells is handled exactly once: as a
    leaf P2P pair, or as one M2L pair of its ancestors at a single level
    (an M2L pair at level l stands for 8^(L-l) x 8^(L-l) leaf pairs)."""
    p2p, m2l = O.pair_counts(L, theta)
    N = (8 << L) ** 3
    covered = p2p + sum(int(m2l[l]) * 8 ** (2 * (L - l)) for l in range(L + 1))
    assert covered == N * (N - 1)
    if L == 0:
        assert p2p + m2l[0] == 512 * 511


def test_pair_counts_golden():
    """Counts stored by tests/golden/make_pair_counts.py (which calls only the
    oracle); guards the rule against silent changes."""
    import json, os
    path = os.path.join(os.path.dirname(__file__), "golden", "pair_counts.json")
    gold = json.load(open(path))
    for key, rec in gold["counts"].items():
        L, theta = rec["L"], rec["theta"]
        if L > 2:
            continue
        p2p, m2l = O.pair_counts(L, theta)
        assert p2p == rec["p2p"] and list(map(int, m2l)) == rec["m2l"], key


# ---------------------------------------------------------------- convergence
def test_convergence_in_order():
    rho = W.sphere_32()["rho"]
    pd, gd = O.direct(rho)
    errs = []
    for p in range(0, 6):
        pf, gf = O.fmm(rho, p=p)
        errs.append((normwise(pf, pd), normwise_vec(gf, gd)))
    for (e0p, e0g), (e1p, e1g) in zip(errs, errs[1:]):
        assert e1p < 0.5 * e0p
        assert e1g < 0.5 * e0g
    # stated accuracy at p = 3, theta = 0.4 on the 32^3 sphere
    assert errs[3][0] < 2e-4 and errs[3][1] < 5e-3


def test_convergence_in_theta():
    rho = W.sphere_32()["rho"]
    pd, gd = O.direct(rho)
    prev = None
    for theta in (0.9, 0.7, 0.5, 0.4):
        pf, gf = O.fmm(rho, theta=theta)
        e = normwise_vec(gf, gd)
        if prev is not None:
            assert e < prev
        prev = e


# ---------------------------------------------------------------- 1/r derivatives
def test_inv_r_derivs_textbook_low_orders():
    R = np.array([0.7, -1.3, 2.1])
    r = np.linalg.norm(R)
    D = O.inv_r_derivs(2, R)
    idx = [tuple(a) for a in O.multi_index(2)]
    assert D[idx.index((0, 0, 0))] == pytest.approx(1 / r, rel=1e-15)
    for k in range(3):
        e = [0, 0, 0]; e[k] = 1
        assert D[idx.index(tuple(e))] == pytest.approx(-R[k] / r ** 3, rel=1e-14)
    for i in range(3):
        for j in range(3):
            a = [0, 0, 0]; a[i] += 1; a[j] += 1
            want = 3 * R[i] * R[j] / r ** 5 - (1.0 if i == j else 0.0) / r ** 3
            assert D[idx.index(tuple(a))] == pytest.approx(want, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("p", [3, 6])
def test_inv_r_derivs_properties(p):
    rng = np.random.default_rng(7)
    idx = [tuple(a) for a in O.multi_index(p)]
    pos = {a: k for k, a in enumerate(idx)}
    for _ in range(5):
        R = rng.normal(size=3) * 2
        D = O.inv_r_derivs(p, R)
        # harmonic: sum_i d^(a + 2 e_i) = 0
        for a in idx:
            if sum(a) + 2 > p:
                continue
            s = sum(D[pos[tuple(np.add(a, 2 * np.eye(3, dtype=int)[i]))]] for i in range(3))
            scale = max(abs(D[pos[tuple(np.add(a, 2 * np.eye(3, dtype=int)[i]))]]) for i in range(3))
            assert abs(s) <= 1e-12 * scale
        # parity and homogeneity
        Dm = O.inv_r_derivs(p, -R)
        D2 = O.inv_r_derivs(p, 2.0 * R)
        for a, k in pos.items():
            n = sum(a)
            assert Dm[k] == pytest.approx((-1) ** n * D[k], rel=1e-13, abs=1e-300)
            assert D2[k] == pytest.approx(2.0 ** (-1 - n) * D[k], rel=1e-13, abs=1e-300)
        # finite differences of one order lower (5-point central, h = 1e-3)
        eps = 1e-3
        for a, k in pos.items():
            if sum(a) + 1 > p:
                continue
            for i in range(3):
                e = np.eye(3)[i] * eps
                f = [O.inv_r_derivs(p, R + s * e)[k] for s in (-2, -1, 1, 2)]
                fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * eps)
                hi = pos[tuple(np.add(a, np.eye(3, dtype=int)[i]))]
                assert fd == pytest.approx(D[hi], rel=1e-7, abs=1e-9 * np.abs(D).max())


# ---------------------------------------------------------------- moments
def test_moments_match_definition():
    """After M2M, M_A^a = sum over the leaves under A of m (x - z_A)^a."""
    rho = W.random_density(16, 51, "signed")
    p = 3
    idx = O.multi_index(p)
    for level in (0, 1):
        M = O.moments(rho, level, p=p)
        nl = 8 << level
        w = 16 // nl                       # leaf cells per level-l cell per axis
        for cell in [(0, 0, 0), (3, 5, 7), (nl - 1, 2, nl - 1)]:
            cx, cy, cz = cell
            zA = (np.array(cell) + 0.5) * w
            sl = rho[cz * w:(cz + 1) * w, cy * w:(cy + 1) * w, cx * w:(cx + 1) * w]
            c = np.arange(w) + 0.5
            zz, yy, xx = np.meshgrid(cz * w + c, cy * w + c, cx * w + c, indexing="ij")
            for k, (t, u, v) in enumerate(idx):
                want = (sl * (xx - zA[0]) ** t * (yy - zA[1]) ** u * (zz - zA[2]) ** v).sum()
                got = M[k, cz, cy, cx]
                assert got == pytest.approx(want, rel=1e-12, abs=1e-12 * np.abs(sl).sum() * w ** 3)


# ---------------------------------------------------------------- adjoint
@pytest.mark.parametrize("n,p", [(8, 3), (16, 3), (16, 5), (32, 3)])
def test_adjoint_dot_product(n, p):
    rng = np.random.default_rng(60 + n + p)
    rho = rng.standard_normal((n, n, n))
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    phi, g = O.fmm(rho, p=p)
    dr = O.fmm_adjoint(w, u, p=p)
    lhs = (w * phi).sum() + (u * g).sum()
    rhs = (dr * rho).sum()
    assert abs(lhs - rhs) / (np.abs(w * phi).sum() + np.abs(u * g).sum()) < 1e-12


def test_adjoint_potential_part_is_forward():
    """With u = 0, d/drho sum(w phi) = h^3 Phi^T w = forward potential of w."""
    rng = np.random.default_rng(71)
    w = rng.standard_normal((16, 16, 16))
    for h in (1.0, 0.25):
        dr = O.fmm_adjoint(w, np.zeros((3, 16, 16, 16)), h=h)
        pw, _ = O.fmm(w, h=h)
        assert normwise(dr, pw) < 1e-12


def test_adjoint_finite_differences():
    rng = np.random.default_rng(81)
    n = 16
    rho = rng.standard_normal((n, n, n))
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    dr = O.fmm_adjoint(w, u)

    def loss(r):
        ph, gg = O.fmm(r)
        return (w * ph).sum() + (u * gg).sum()

    for j in rng.choice(n ** 3, 6, replace=False):
        for eps, tol in ((1.0, 1e-10), (1e-3, 1e-7)):
            e = np.zeros(n ** 3); e[j] = eps
            e = e.reshape(n, n, n)
            fd = (loss(rho + e) - loss(rho - e)) / (2 * eps)
            assert fd == pytest.approx(dr.reshape(-1)[j], rel=tol, abs=tol * np.abs(dr).max())


# ---------------------------------------------------------------- variants
def test_slab_and_sink_variants_agree_with_full():
    rng = np.random.default_rng(91)
    n = 32
    rho = rng.standard_normal((n, n, n))
    phi, g = O.fmm(rho)
    ps, gs = O.fmm(rho, zslab=(8, 13))
    assert np.array_equal(ps[8:13], phi[8:13]) and np.array_equal(gs[:, 8:13], g[:, 8:13])
    assert not ps[:8].any() and not ps[13:].any()
    sk = rng.choice(n ** 3, 40, replace=False)
    pk, gk = O.fmm_sinks(rho, sk)
    assert np.abs(pk - phi.reshape(-1)[sk]).max() < 1e-13 * np.abs(phi).max()
    assert np.abs(gk - g.reshape(3, -1)[:, sk]).max() < 1e-13 * np.abs(g).max()
    w = rng.standard_normal((n, n, n)); u = rng.standard_normal((3, n, n, n))
    dr = O.fmm_adjoint(w, u)
    ds = O.fmm_adjoint(w, u, zslab=(20, 32))
    assert np.array_equal(ds[20:], dr[20:])


def test_direct_sampled_sinks_match_full():
    rho = W.random_density(16, 95, "uniform")
    phi, g = O.direct(rho)
    sk = np.array([0, 17, 4095, 2048])
    ps, gs = O.direct(rho, sinks=sk)
    assert np.array_equal(ps, phi.reshape(-1)[sk])
    assert np.array_equal(gs, g.reshape(3, -1)[:, sk])


# ---------------------------------------------------------------- inputs
def test_lane_emden_first_zero_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "lane_emden_n1.5.txt")
    xi1 = [float(l.split()[1]) for l in open(path) if l.startswith("xi_1")][0]
    _, _, got = W.lane_emden(1.5)
    assert got == pytest.approx(xi1, abs=5e-6)
