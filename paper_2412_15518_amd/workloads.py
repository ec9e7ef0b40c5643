"""Seeded synthetic inputs: octree layouts of 8^3-cell sub-grids and densities.

This module holds no arithmetic of the fast multipole method.  It serves both
the GPU library's callers and the tests' CPU oracle, so both see bit-identical
inputs.

The paper runs on production restart files of a double-white-dwarf merger (Sec.
6.1, table "tab:data:set") that are not public in a usable form here; the
densities below stand in for them with the same structure: a uniform sphere, two
n = 1.5 polytropes on a tenuous floor, and lognormal noise inside a sphere.

Dense grids are numpy arrays of shape (n, n, n) indexed [z, y, x] (x fastest).
The library's own layout is sub-grid-major: leaf k of the layout owns the 512
values [512 k, 512 k + 512), x fastest inside the sub-grid (Sec. 4.3: each tree
node holds an 8x8x8 sub-grid).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SUBGRID = 8          # cells per axis of one tree node (Sec. 4.3)


# --------------------------------------------------------------------------
# octree layouts
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Layout:
    """An octree of 8^3 sub-grids in the form the C-ABI takes.

    level[i], coord[i] (sub-grid coordinates at that level), parent[i] (-1 for
    the root, which is node 0) and is_leaf[i] for each node i.
    """
    level: np.ndarray      # int32 [n_nodes]
    coord: np.ndarray      # int32 [n_nodes, 3]  (x, y, z)
    parent: np.ndarray     # int32 [n_nodes]
    is_leaf: np.ndarray    # uint8 [n_nodes]
    h_leaf_min: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)
    G: float = 1.0

    @property
    def n_nodes(self) -> int:
        return int(self.level.shape[0])

    @property
    def leaf_nodes(self) -> np.ndarray:
        """Node ids of the leaves, in layout order (the order of rho's blocks)."""
        return np.nonzero(self.is_leaf)[0]

    @property
    def depth(self) -> int:
        return int(self.level.max())

    @property
    def n_leaf_cells(self) -> int:
        return int(self.is_leaf.sum()) * SUBGRID ** 3

    def is_uniform(self) -> bool:
        L = self.depth
        return bool(np.all(self.level[self.is_leaf.astype(bool)] == L))

    # permutations between a dense grid (uniform trees) and layout order
    def _leaf_index(self) -> np.ndarray:
        if not self.is_uniform():
            raise ValueError("dense <-> layout conversion needs a uniform tree")
        L = self.depth
        n = SUBGRID << L
        leaves = self.leaf_nodes
        c = self.coord[leaves].astype(np.int64)                 # [nleaf, 3]
        l = np.arange(SUBGRID, dtype=np.int64)
        lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")        # local cell, x fastest
        gx = c[:, 0, None, None, None] * SUBGRID + lx
        gy = c[:, 1, None, None, None] * SUBGRID + ly
        gz = c[:, 2, None, None, None] * SUBGRID + lz
        return ((gz * n + gy) * n + gx).reshape(-1)             # layout pos -> dense idx

    def dense_to_layout(self, a: np.ndarray) -> np.ndarray:
        """(…, n, n, n) dense -> (…, n_leaf_cells) in layout order."""
        idx = self._leaf_index()
        flat = a.reshape(a.shape[:-3] + (-1,))
        return np.ascontiguousarray(flat[..., idx])

    def layout_to_dense(self, a: np.ndarray) -> np.ndarray:
        """(…, n_leaf_cells) in layout order -> (…, n, n, n) dense."""
        idx = self._leaf_index()
        n = SUBGRID << self.depth
        out = np.empty(a.shape[:-1] + (n ** 3,), dtype=a.dtype)
        out[..., idx] = a
        return out.reshape(a.shape[:-1] + (n, n, n))


def _morton_key(c: np.ndarray) -> np.ndarray:
    key = np.zeros(c.shape[0], dtype=np.int64)
    for bit in range(16):
        for ax in range(3):
            key |= ((c[:, ax].astype(np.int64) >> bit) & 1) << (3 * bit + ax)
    return key


def uniform_layout(L: int, order: str = "lex", seed: int | None = None,
                   h: float = 1.0, G: float = 1.0) -> Layout:
    """Full octree of depth L: every node at levels < L has 8 children, the
    leaves are the 8^L nodes at level L; the leaf grid is (8*2^L)^3 cells.

    order: "lex" (z, y, x), "morton", or "random" (a seeded shuffle of all
    non-root nodes, which exercises the layout-order mapping).
    """
    if L < 0:
        raise ValueError("L must be >= 0")
    levels, coords = [], []
    for l in range(L + 1):
        m = 1 << l
        g = np.arange(m, dtype=np.int32)
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        c = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
        if order == "morton":
            c = c[np.argsort(_morton_key(c), kind="stable")]
        levels.append(np.full(c.shape[0], l, dtype=np.int32))
        coords.append(c)
    level = np.concatenate(levels)
    coord = np.concatenate(coords).astype(np.int32)
    if order == "random":
        rng = np.random.default_rng(seed)
        perm = np.concatenate([[0], 1 + rng.permutation(level.shape[0] - 1)])
        level, coord = level[perm], coord[perm]
    elif order not in ("lex", "morton"):
        raise ValueError(f"unknown order {order!r}")
    # parents by coordinate lookup
    pos = {(int(l), int(c[0]), int(c[1]), int(c[2])): i for i, (l, c) in enumerate(zip(level, coord))}
    parent = np.full(level.shape[0], -1, dtype=np.int32)
    for i, (l, c) in enumerate(zip(level, coord)):
        if l > 0:
            parent[i] = pos[(int(l) - 1, int(c[0]) >> 1, int(c[1]) >> 1, int(c[2]) >> 1)]
    is_leaf = (level == L).astype(np.uint8)
    return Layout(level=level, coord=coord, parent=parent, is_leaf=is_leaf, h_leaf_min=h, G=G)


# --------------------------------------------------------------------------
# densities (dense grids, cell centres at (c + 1/2) h)
# --------------------------------------------------------------------------
def _centre_r(n: int, centre, h: float = 1.0) -> np.ndarray:
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)


def uniform_sphere(n: int, radius: float, centre=None, value: float = 1.0) -> np.ndarray:
    """value where the cell centre lies within `radius` of `centre` (<=), else 0."""
    if centre is None:
        centre = (n / 2.0,) * 3
    return np.where(_centre_r(n, centre) <= radius, value, 0.0).astype(np.float64)


def lane_emden(n_index: float = 1.5, dxi: float = 1e-4):
    """theta(xi) of the Lane-Emden equation theta'' + 2 theta'/xi + theta^n = 0
    (theta(0) = 1, theta'(0) = 0) by classical RK4 up to the first zero xi_1.
    Returns (xi_grid, theta_grid, xi_1)."""
    xi = 1e-6
    y = np.array([1.0 - xi * xi / 6.0, -xi / 3.0])

    def f(x, v):
        return np.array([v[1], -max(v[0], 0.0) ** n_index - 2.0 * v[1] / x])

    xs, ts = [0.0, xi], [1.0, y[0]]
    while True:
        k1 = f(xi, y)
        k2 = f(xi + dxi / 2, y + dxi / 2 * k1)
        k3 = f(xi + dxi / 2, y + dxi / 2 * k2)
        k4 = f(xi + dxi, y + dxi * k3)
        ynew = y + dxi / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if ynew[0] <= 0.0:
            xi1 = xi + dxi * y[0] / (y[0] - ynew[0])
            xs.append(xi1)
            ts.append(0.0)
            return np.array(xs), np.array(ts), xi1
        y = ynew
        xi += dxi
        xs.append(xi)
        ts.append(y[0])


_LE_CACHE: dict = {}


def polytrope(n: int, centre, radius: float, rho_c: float, n_index: float = 1.5) -> np.ndarray:
    """rho_c * theta(xi)^n_index with xi = xi_1 r / radius inside the star, 0 outside."""
    if n_index not in _LE_CACHE:
        _LE_CACHE[n_index] = lane_emden(n_index)
    xs, ts, xi1 = _LE_CACHE[n_index]
    r = _centre_r(n, centre)
    inside = r <= radius
    theta = np.interp(np.where(inside, xi1 * r / radius, 0.0), xs, ts)
    return np.where(inside, rho_c * np.maximum(theta, 0.0) ** n_index, 0.0)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def sphere_32():
    """32^3 (L = 2): rho = 1 for centres within 12 of the box centre, else 0."""
    return dict(L=2, rho=uniform_sphere(32, 12.0, (16.0, 16.0, 16.0)))


def two_polytropes(n: int = 128, seed: int = 2, with_cotangents: bool = True):
    """128^3 (L = 4): two n = 1.5 polytropes (rho_c 1.0, R 20 at x = 39; rho_c 0.6,
    R 14 at x = 89; y = z = 64), a 1e-10 floor, and x(1 + 0.01 U(-1,1)) noise.
    The cotangents w, u ~ N(0,1) for the forward+adjoint pass follow from the
    same generator.  Other n scale the geometry by n/128."""
    s = n / 128.0
    rng = np.random.default_rng(seed)
    rho = (polytrope(n, (39 * s, 64 * s, 64 * s), 20 * s, 1.0)
           + polytrope(n, (89 * s, 64 * s, 64 * s), 14 * s, 0.6)
           + 1e-10)
    rho = rho * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=rho.shape))
    L = int(round(math.log2(n // SUBGRID)))
    out = dict(L=L, rho=rho)
    if with_cotangents:
        out["w"] = rng.standard_normal((n, n, n))
        out["u"] = rng.standard_normal((3, n, n, n))
    return out


def lognormal_sphere(n: int = 64, seed: int = 5, n_fd: int = 64):
    """64^3 (L = 3): rho = exp(0.5 z) * [r <= 24] about the box centre with
    z ~ N(0,1); cotangents w, u ~ N(0,1); n_fd distinct finite-difference
    cells.  Drawn in the fixed order rho, w, u, cells."""
    rng = np.random.default_rng(seed)
    rad = 24.0 * n / 64.0
    rho = np.exp(0.5 * rng.standard_normal((n, n, n))) * uniform_sphere(n, rad, (n / 2.0,) * 3)
    w = rng.standard_normal((n, n, n))
    u = rng.standard_normal((3, n, n, n))
    cells = rng.choice(n ** 3, size=n_fd, replace=False).astype(np.int64)
    L = int(round(math.log2(n // SUBGRID)))
    return dict(L=L, rho=rho, w=w, u=u, cells=cells)


def batch_of_octrees(count: int = 16, seed: int = 3, lo: int = 64, hi: int = 1024, Lcap: int = 4):
    """Independent adaptive octrees for the batched path.  Leaf sub-grid targets
    are drawn log-uniform in [lo, hi]; each tree holds a uniform sphere or an
    n = 1.5 polytrope (random centre, radius, rho_c) on a 1e-10 floor in a box of
    8 * 2^Lcap cells of the deepest allowed level, and grows from its root by
    density-ranked refinement: each round refines the leaves of highest peak
    density at their cell centres (ties: coarser level, then nearer the star's
    centre), then balances the tree 2:1, until the leaf count reaches the
    target.  rho (at the leaf cell centres) and cotangents w, u ~ N(0,1) are in
    layout order.  Drawn in the order: targets, then per tree kind, centre,
    radius, rho_c, w, u."""
    rng = np.random.default_rng(seed)
    counts = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))
    box = float(SUBGRID << Lcap)
    l8 = np.arange(SUBGRID, dtype=np.float64)
    lz, ly, lx = np.meshgrid(l8, l8, l8, indexing="ij")
    loc = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], axis=1) + 0.5
    trees = []
    for c in counts:
        target = int(round(c))
        kind = "sphere" if rng.uniform() < 0.5 else "polytrope"
        centre = rng.uniform(0.3 * box, 0.7 * box, size=3)
        radius = float(rng.uniform(0.15 * box, 0.35 * box))
        rho_c = float(rng.uniform(0.5, 1.0))

        def rho_at(pts, kind=kind, centre=centre, radius=radius, rho_c=rho_c):
            if kind == "sphere":
                r = np.sqrt(((pts - centre) ** 2).sum(axis=-1))
                return np.where(r <= radius, rho_c, 0.0) + 1e-10
            return _polytrope_at(pts, centre, radius, rho_c) + 1e-10

        refined = [set() for _ in range(Lcap)]
        leaves = [(0, (0, 0, 0))]
        while len(leaves) < target:
            cand = [(l, q) for (l, q) in leaves if l < Lcap]
            if not cand:
                break
            lv = np.array([l for l, _ in cand], dtype=np.float64)
            cq = np.array([q for _, q in cand], dtype=np.float64)
            hl = 2.0 ** (Lcap - lv)
            pts = (cq[:, None, :] * SUBGRID + loc[None]) * hl[:, None, None]
            peak = rho_at(pts).max(axis=1)
            dist = np.sqrt((((cq + 0.5) * SUBGRID * hl[:, None] - centre) ** 2).sum(axis=1))
            order = np.lexsort((dist, lv, -peak))
            k = max(1, int(math.ceil((target - len(leaves)) / 14.0)))
            for i in order[:k]:
                refined[int(lv[i])].add(tuple(int(v) for v in cq[i]))
            _balance(refined, Lcap)
            lay = _layout_of(refined, Lcap, 1.0, 1.0)
            leaves = [(int(lay.level[i]), tuple(int(v) for v in lay.coord[i])) for i in lay.leaf_nodes]
        lay = _layout_of(refined, Lcap, 1.0, 1.0)
        centres, _ = leaf_cell_centres(lay)        # box units: the tree's h_leaf_min is 2^(Lcap - depth)
        rho = rho_at(centres)
        w = rng.standard_normal(lay.n_leaf_cells)
        u = rng.standard_normal((3, lay.n_leaf_cells))
        trees.append(dict(layout=lay, kind=kind, leaf_count=float(c), target=target,
                          n_leaf=int(lay.is_leaf.sum()), rho=rho, w=w, u=u))
    return trees


def random_density(n: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Plain random fields for small parity cases."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(0.0, 1.0, size=(n, n, n))
    if kind == "signed":
        return rng.standard_normal((n, n, n))
    if kind == "sparse":
        a = np.zeros(n ** 3)
        k = max(1, n ** 3 // 50)
        a[rng.choice(n ** 3, size=k, replace=False)] = rng.uniform(0.5, 2.0, size=k)
        return a.reshape(n, n, n)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# adaptive octrees
# --------------------------------------------------------------------------
_NEIGHBOURS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
               if (dx, dy, dz) != (0, 0, 0)]


def _balance(refined: list, Lmax: int) -> None:
    """2:1 balance in place: wherever a node of level l is refined, the 26
    nodes around it at level l must exist, so their parents are refined (and
    so on up the levels)."""
    changed = True
    while changed:
        changed = False
        for l in range(Lmax - 1, 0, -1):
            m = 1 << l
            for (x, y, z) in list(refined[l]):
                for dx, dy, dz in _NEIGHBOURS:
                    q = (x + dx, y + dy, z + dz)
                    if min(q) < 0 or max(q) >= m:
                        continue
                    par = (q[0] >> 1, q[1] >> 1, q[2] >> 1)
                    if par not in refined[l - 1]:
                        refined[l - 1].add(par)
                        changed = True


def _layout_of(refined: list, Lmax: int, h: float, G: float) -> Layout:
    """The octree whose refined nodes per level are `refined` (every refined
    node's parent refined), listed level by level, z-major inside a level."""
    levels, coords, leaf = [], [], []
    cur = [(0, 0, 0)]
    for l in range(Lmax + 1):
        cur = sorted(cur, key=lambda c: (c[2], c[1], c[0]))
        for c in cur:
            levels.append(l)
            coords.append(c)
            leaf.append(l == Lmax or c not in refined[l])
        if l < Lmax:
            cur = [(2 * x + (b & 1), 2 * y + ((b >> 1) & 1), 2 * z + (b >> 2))
                   for (x, y, z) in cur if (x, y, z) in refined[l] for b in range(8)]
    depth = max([l for l in range(Lmax) if refined[l]], default=-1) + 1
    level = np.array(levels, dtype=np.int32)
    coord = np.array(coords, dtype=np.int32).reshape(-1, 3)
    keep = level <= depth
    level, coord = level[keep], coord[keep]
    is_leaf = np.array(leaf, dtype=np.uint8)[keep]
    is_leaf[level == depth] = 1
    pos = {(int(l), int(c[0]), int(c[1]), int(c[2])): i for i, (l, c) in enumerate(zip(level, coord))}
    parent = np.full(level.shape[0], -1, dtype=np.int32)
    for i, (l, c) in enumerate(zip(level, coord)):
        if l > 0:
            parent[i] = pos[(int(l) - 1, int(c[0]) >> 1, int(c[1]) >> 1, int(c[2]) >> 1)]
    return Layout(level=level, coord=coord, parent=parent, is_leaf=is_leaf,
                  h_leaf_min=h * 2.0 ** (Lmax - depth), G=G)


def adaptive_layout(Lmax: int, refine, base: int = 0, h: float = 1.0, G: float = 1.0) -> Layout:
    """Octree refined top-down: every node above level `base` is refined, and a
    node of level l in [base, Lmax) is refined where refine(l, coords) says so
    (coords: int array [k, 3] of sub-grid coordinates; returns bool [k]).  The
    tree is then balanced 2:1: wherever a node of level l is refined, the 26
    nodes around it at level l exist (refining their parents as needed), so
    leaf sub-grids that touch lie at most one level apart.  Nodes are listed
    level by level, z-major inside a level; h is the cell width of level Lmax
    (the tree's own finest level may be coarser)."""
    if Lmax < 0 or not 0 <= base <= Lmax:
        raise ValueError("need 0 <= base <= Lmax")
    refined = [set() for _ in range(Lmax)]
    nodes = {(0, 0, 0)}
    for l in range(Lmax):
        cur = sorted(nodes)
        arr = np.array(cur, dtype=np.int64).reshape(-1, 3)
        want = np.ones(len(cur), dtype=bool) if l < base else np.asarray(refine(l, arr), dtype=bool)
        refined[l] = {c for c, w in zip(cur, want) if w}
        nodes = {(2 * x + (b & 1), 2 * y + ((b >> 1) & 1), 2 * z + (b >> 2))
                 for (x, y, z) in refined[l] for b in range(8)}
    _balance(refined, Lmax)
    return _layout_of(refined, Lmax, h, G)


def leaf_cell_centres(layout: Layout) -> tuple:
    """(centres [n_leaf_cells, 3], cell widths [n_leaf_cells]) in layout order,
    for a tree whose finest level has cell width layout.h_leaf_min."""
    Lmax = layout.depth
    leaves = layout.leaf_nodes
    l = np.arange(SUBGRID, dtype=np.int64)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    loc = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], axis=1)                 # [512, 3]
    hl = layout.h_leaf_min * (2.0 ** (Lmax - layout.level[leaves].astype(np.float64)))
    cells = layout.coord[leaves].astype(np.int64)[:, None, :] * SUBGRID + loc[None]
    centres = (cells + 0.5) * hl[:, None, None]
    return centres.reshape(-1, 3), np.repeat(hl, SUBGRID ** 3)


def _polytrope_at(points: np.ndarray, centre, radius: float, rho_c: float, n_index: float = 1.5):
    if n_index not in _LE_CACHE:
        _LE_CACHE[n_index] = lane_emden(n_index)
    xs, ts, xi1 = _LE_CACHE[n_index]
    r = np.sqrt(((points - np.asarray(centre, dtype=np.float64)) ** 2).sum(axis=-1))
    inside = r <= radius
    theta = np.interp(np.where(inside, xi1 * r / radius, 0.0), xs, ts)
    return np.where(inside, rho_c * np.maximum(theta, 0.0) ** n_index, 0.0)


def adaptive_two_polytropes(seed: int = 3, base: int = 3, extra: int = 3, thresh: float = 1e-3,
             with_cotangents: bool = True):
    """Adaptive octree over a box of (8 * 2^(base + extra))^3 finest cells
    (h = 1): uniform down to level `base`, then refined `extra` more levels
    wherever a cell centre of the sub-grid has rho > thresh * rho_peak, and
    balanced 2:1.  rho: the two n = 1.5 polytropes of the 128^3 workload at the
    same sizes in finest cells (rho_c 1.0, R 20 and rho_c 0.6, R 14, centres 50
    apart along x about the box centre) plus a 1e-10 floor, evaluated at the
    leaf cell centres, times (1 + 0.01 U(-1,1)) drawn in layout order;
    cotangents w, u ~ N(0,1) per leaf cell follow."""
    Lmax = base + extra
    nbox = SUBGRID << Lmax
    c0 = nbox / 2.0
    stars = [((c0 - 25.0, c0, c0), 20.0, 1.0), ((c0 + 25.0, c0, c0), 14.0, 0.6)]
    floor = 1e-10
    peak = 1.0 + floor

    def rho_at(pts):
        out = np.full(pts.shape[:-1], floor)
        for ctr, rad, rc in stars:
            out = out + _polytrope_at(pts, ctr, rad, rc)
        return out

    l = np.arange(SUBGRID, dtype=np.float64)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    loc = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], axis=1)

    def refine(level, coords):
        hl = float(2 ** (Lmax - level))
        pts = (coords[:, None, :] * SUBGRID + loc[None] + 0.5) * hl
        return (rho_at(pts) > thresh * peak).any(axis=1)

    layout = adaptive_layout(Lmax, refine, base=base)
    rng = np.random.default_rng(seed)
    centres, _ = leaf_cell_centres(layout)
    rho = rho_at(centres) * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=centres.shape[0]))
    out = dict(layout=layout, rho=rho, Lmax=Lmax)
    if with_cotangents:
        out["w"] = rng.standard_normal(centres.shape[0])
        out["u"] = rng.standard_normal((3, centres.shape[0]))
    return out


def small_amr(kind: str = "corner", seed: int = 7):
    """Small adaptive trees for parity cases, with rho ~ U(0.5, 1.5) per leaf
    cell (seeded, layout order).  'corner': depth 2, one level-1 node refined
    (7 + 8 leaves); 'blob': depth 3 refined around an off-centre point (the
    balance refines all of level 1; leaves on levels 2 and 3); 'edge': depth 3 refined along a box edge, so
    the balance reaches the domain boundary."""
    if kind == "corner":
        lay = adaptive_layout(2, lambda l, c: (c == 0).all(axis=1), base=1)
    elif kind == "blob":
        p = np.array([2.2, 5.1, 3.4])
        lay = adaptive_layout(3, lambda l, c: np.linalg.norm((c + 0.5) / (1 << l) * 8 - p, axis=1) < 8.0 / (1 << l) * 1.2,
                              base=1)
    elif kind == "edge":
        lay = adaptive_layout(3, lambda l, c: (c[:, 0] == 0) & (c[:, 1] == 0) & (c[:, 2] <= 1), base=1)
    else:
        raise ValueError(kind)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, size=lay.n_leaf_cells)
    return dict(layout=lay, rho=rho)
