"""Plain FP64 CPU oracle for the octree FMM gravity solve (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product library.  It shares no code
with the GPU path; the C source is otfmm_oracle.c next to this file.

All grids are dense numpy float64 arrays of shape (n, n, n) indexed [z, y, x];
accelerations are (3, n, n, n).  Leaf level L gives n = 8 * 2^L.  The method's
readings (opening rule, expansion centres, total-order truncation) are those of
the C source's header.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = C.CDLL(_build.LIB)
    lib.oracle_ncomp.argtypes = [C.c_int]
    lib.oracle_threads.argtypes = []
    lib.oracle_multi_index.argtypes = [C.c_int, _ip]
    lib.oracle_inv_r_derivs.argtypes = [C.c_int, _dp, _dp]
    lib.oracle_direct.argtypes = [C.c_int, C.c_double, C.c_double, _dp, C.c_int64, _i64p, _dp, _dp]
    lib.oracle_fmm.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
    lib.oracle_fmm_slab.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                    C.c_int, C.c_int, _dp, _dp]
    lib.oracle_fmm_sinks.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                     C.c_int64, _i64p, _dp, _dp]
    lib.oracle_fmm_adjoint.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                       _dp, _dp, _dp]
    lib.oracle_fmm_adjoint_slab.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                            _dp, _dp, C.c_int, C.c_int, _dp]
    lib.oracle_moments.argtypes = [C.c_int, C.c_int, C.c_double, _dp, C.c_int, _dp]
    lib.oracle_pair_counts.argtypes = [C.c_int, C.c_double, _i64p, _i64p]
    lib.oracle_pair_counts_slab.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _i64p, _i64p]
    lib.oracle_amcorr_sinks.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                        C.c_int64, _i64p, _dp]
    _tree = [C.c_int64, _i32p, _i32p, _u8p]
    lib.oracle_amr_sinks.argtypes = _tree + [C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                             C.c_int64, _i64p, _dp, _dp]
    lib.oracle_amr_direct.argtypes = _tree + [C.c_double, C.c_double, _dp, C.c_int64, _i64p, _dp, _dp]
    lib.oracle_amr_cover.argtypes = _tree + [C.c_double, C.c_int64, _i32p]
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _level_of(rho) -> int:
    n = rho.shape[-1]
    L = int(round(np.log2(n / 8)))
    if rho.shape[-3:] != (n, n, n) or (8 << L) != n:
        raise ValueError(f"grid must be (n,n,n) with n = 8*2^L, got {rho.shape}")
    return L


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed (rc={rc})")


def ncomp(p: int) -> int:
    return int(_load().oracle_ncomp(p))


def threads() -> int:
    return int(_load().oracle_threads())


def multi_index(p: int) -> np.ndarray:
    out = np.zeros((ncomp(p), 3), dtype=np.int32)
    _check(_load().oracle_multi_index(p, out.ctypes.data_as(_ip)), "multi_index")
    return out


def inv_r_derivs(p: int, R) -> np.ndarray:
    """Derivatives d^a (1/r) at R for all |a| <= p (order of multi_index(p))."""
    R = _c64(R)
    out = np.zeros(ncomp(p))
    _check(_load().oracle_inv_r_derivs(p, _d(R), _d(out)), "inv_r_derivs")
    return out


def direct(rho, h=1.0, G=1.0, sinks=None):
    """Direct Newtonian sum over cell centres (i != j).  sinks: None for the
    whole grid (returns dense phi, g), or dense cell indices (returns per sink)."""
    rho = _c64(rho)
    n = rho.shape[-1]
    lib = _load()
    if sinks is None:
        phi = np.zeros((n, n, n)); g = np.zeros((3, n, n, n))
        _check(lib.oracle_direct(n, h, G, _d(rho), 0, None, _d(phi), _d(g)), "direct")
        return phi, g
    s = np.ascontiguousarray(sinks, dtype=np.int64)
    phi = np.zeros(s.size); g = np.zeros((3, s.size))
    _check(lib.oracle_direct(n, h, G, _d(rho), s.size, s.ctypes.data_as(_i64p), _d(phi), _d(g)), "direct")
    return phi, g


def fmm(rho, p=3, theta=0.4, h=1.0, G=1.0, zslab=None):
    """FMM forward; with zslab=(zlo, zhi) only leaves of that z-slab are computed
    (the rest of phi, g stays 0)."""
    rho = _c64(rho)
    L = _level_of(rho)
    n = rho.shape[-1]
    phi = np.zeros((n, n, n)); g = np.zeros((3, n, n, n))
    zlo, zhi = (0, n) if zslab is None else zslab
    _check(_load().oracle_fmm_slab(L, p, theta, h, G, _d(rho), zlo, zhi, _d(phi), _d(g)), "fmm")
    return phi, g


def fmm_sinks(rho, sinks, p=3, theta=0.4, h=1.0, G=1.0):
    """FMM forward at selected leaf cells (dense indices), evaluated per sink."""
    rho = _c64(rho)
    L = _level_of(rho)
    s = np.ascontiguousarray(sinks, dtype=np.int64)
    phi = np.zeros(s.size); g = np.zeros((3, s.size))
    _check(_load().oracle_fmm_sinks(L, p, theta, h, G, _d(rho), s.size, s.ctypes.data_as(_i64p),
                                    _d(phi), _d(g)), "fmm_sinks")
    return phi, g


def fmm_adjoint(w, u, p=3, theta=0.4, h=1.0, G=1.0, zslab=None):
    """d/d rho of sum(w * phi) + sum(u * g) through the FMM (transposed chain)."""
    w = _c64(w); u = _c64(u)
    L = _level_of(w)
    n = w.shape[-1]
    if u.shape != (3, n, n, n):
        raise ValueError("u must be (3, n, n, n)")
    drho = np.zeros((n, n, n))
    zlo, zhi = (0, n) if zslab is None else zslab
    _check(_load().oracle_fmm_adjoint_slab(L, p, theta, h, G, _d(w), _d(u), zlo, zhi, _d(drho)),
           "fmm_adjoint")
    return drho


def moments(rho, level, p=3, h=1.0):
    """Moments M^a (no factorial, about geometric centres) of every cell of
    `level` after the upward pass: array (ncomp, n_l, n_l, n_l)."""
    rho = _c64(rho)
    L = _level_of(rho)
    nl = 8 << level
    out = np.zeros((ncomp(p), nl, nl, nl))
    _check(_load().oracle_moments(L, p, h, _d(rho), level, _d(out)), "moments")
    return out


def pair_counts(L, theta=0.4, zslab=None):
    """(p2p, m2l[0..L]) ordered-pair counts by brute-force enumeration."""
    m2l = np.zeros(L + 1, dtype=np.int64)
    p2p = C.c_int64(0)
    n = 8 << L
    zlo, zhi = (0, n) if zslab is None else zslab
    _check(_load().oracle_pair_counts_slab(L, theta, zlo, zhi, C.byref(p2p), m2l.ctypes.data_as(_i64p)),
           "pair_counts")
    return int(p2p.value), m2l


# --------------------------------------------------------------------------
# adaptive octrees: layouts as in the library (level, coord [n, 3], is_leaf),
# leaf-cell arrays in layout order (512 per leaf sub-grid, x fastest)
# --------------------------------------------------------------------------
def _tree_args(layout):
    lvl = np.ascontiguousarray(layout.level, dtype=np.int32)
    crd = np.ascontiguousarray(layout.coord, dtype=np.int32)
    leaf = np.ascontiguousarray(layout.is_leaf, dtype=np.uint8)
    keep = (lvl, crd, leaf)
    return keep, [lvl.shape[0], lvl.ctypes.data_as(_i32p), crd.ctypes.data_as(_i32p), leaf.ctypes.data_as(_u8p)]


def _sinks(layout, sinks):
    n = int(layout.is_leaf.sum()) * 512
    return np.arange(n, dtype=np.int64) if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)


def amr_fmm_sinks(layout, rho, sinks=None, p=3, theta=0.4, G=None):
    """FMM forward on an adaptive octree at the given leaf cells (all when
    None): (phi [k], g [3, k]).  Raises on trees that are not 2:1 balanced."""
    keep, t = _tree_args(layout)
    rho = _c64(rho)
    s = _sinks(layout, sinks)
    phi = np.zeros(s.size); g = np.zeros((3, s.size))
    G = layout.G if G is None else G
    rc = _load().oracle_amr_sinks(*t, p, theta, layout.h_leaf_min, G, _d(rho), s.size,
                                  s.ctypes.data_as(_i64p), _d(phi), _d(g))
    _check(rc, "amr_fmm_sinks")
    return phi, g


def amr_direct(layout, rho, sinks=None, G=None):
    """Direct sum over all leaf cells (point masses rho h_l^3 at the centres)."""
    keep, t = _tree_args(layout)
    rho = _c64(rho)
    s = _sinks(layout, sinks)
    phi = np.zeros(s.size); g = np.zeros((3, s.size))
    G = layout.G if G is None else G
    _check(_load().oracle_amr_direct(*t, layout.h_leaf_min, G, _d(rho), s.size, s.ctypes.data_as(_i64p),
                                     _d(phi), _d(g)), "amr_direct")
    return phi, g


def amr_cover(layout, sink, theta=0.4):
    """How many times the partners of leaf cell `sink` account for each leaf cell."""
    keep, t = _tree_args(layout)
    mult = np.zeros(int(layout.is_leaf.sum()) * 512, dtype=np.int32)
    _check(_load().oracle_amr_cover(*t, theta, int(sink), mult.ctypes.data_as(_i32p)), "amr_cover")
    return mult


def am_correction(rho, p=3, theta=0.4, h=1.0, G=1.0, sinks=None):
    """Spin torque per unit mass t (3, ...) of the angular-momentum correction:
    sum_i m_i (x_i x g_i + t_i) = 0 for the FMM's g (uniform trees).  sinks:
    None for the whole grid (dense (3, n, n, n)), else dense cell indices."""
    rho = _c64(rho)
    L = _level_of(rho)
    n = rho.shape[-1]
    s = np.arange(n ** 3, dtype=np.int64) if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    t = np.zeros((3, s.size))
    _check(_load().oracle_amcorr_sinks(L, p, theta, h, G, _d(rho), s.size, s.ctypes.data_as(_i64p), _d(t)),
           "amcorr_sinks")
    return t.reshape(3, n, n, n) if sinks is None else t
