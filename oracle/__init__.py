"""FP64 CPU oracle for the GreeM short-range tree force -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.
The HIP library never loads it and shares no code with it.

``oracle/treepm_oracle.c`` (built into ``liboracle.so`` by ``oracle/build.py``) holds the pair
law of eq. (1)-(2), the exact short-range direct sums and the reference tree/walk/list force.
``oracle/ewald.py`` holds the tiny-N periodic Ewald sum and the Fourier long-range part used
to pin the cutoff function as the complement of the PM force.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# A test may point this at a deliberately broken build of the oracle (mutation checks).
LIB_PATH = os.environ.get("TREEPM_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

_lib = None

_d = C.c_double
_i64 = C.c_int64
_p = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.orc_g_p3m.restype = _d
        L.orc_g_p3m.argtypes = [_d]
        L.orc_pair.restype = None
        L.orc_pair.argtypes = [_p, _p, _d, _d, _d, _d, _p]
        for name in ("orc_direct_brute", "orc_direct_cells"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [_i64, _p, _p, _p, _p, _d, _d, _d, _p, _p, _p, C.c_int]
        L.orc_tree_build.restype = _p
        L.orc_tree_build.argtypes = [_i64, _p, _p, _p, _p, _d, _d, _d, _d, C.c_int, C.c_int]
        L.orc_tree_free.restype = None
        L.orc_tree_free.argtypes = [_p]
        L.orc_tree_walk.restype = _i64
        L.orc_tree_walk.argtypes = [_p]
        L.orc_tree_force.restype = C.c_int
        L.orc_tree_force.argtypes = [_p, _p, _p, _p, C.c_int]
        L.orc_tree_force_mag.restype = C.c_int
        L.orc_tree_force_mag.argtypes = [_p, _p, _p, C.c_int]
        L.orc_tree_walk_force_sample.restype = _i64
        L.orc_tree_walk_force_sample.argtypes = [_p, _i64, _i64, _p, _p, _p, C.c_int, _p, _p,
                                                 _p]
        for name in ("orc_tree_n_nodes", "orc_tree_n_groups", "orc_tree_n_entries",
                     "orc_tree_interactions"):
            f = getattr(L, name)
            f.restype = _i64
            f.argtypes = [_p]
        L.orc_tree_sorted.restype = None
        L.orc_tree_sorted.argtypes = [_p, _p, _p]
        L.orc_tree_nodes.restype = None
        L.orc_tree_nodes.argtypes = [_p] + [_p] * 8
        L.orc_tree_groups.restype = None
        L.orc_tree_groups.argtypes = [_p] * 7
        L.orc_tree_lists.restype = C.c_int
        L.orc_tree_lists.argtypes = [_p, _p, _p, _p]
        L.orc_theta_r.restype = _d
        L.orc_theta_r.argtypes = [_d, _d, _d, _d]
        L.orc_tree_set_opening.restype = C.c_int
        L.orc_tree_set_opening.argtypes = [_p, C.c_int, _d]
        L.orc_tree_set_theta.restype = C.c_int
        L.orc_tree_set_theta.argtypes = [_p, _d]
        L.orc_g_p3m_derivs.restype = None
        L.orc_g_p3m_derivs.argtypes = [_d, _p, _p]
        L.orc_cell_acc.restype = None
        L.orc_cell_acc.argtypes = [_p, _p, _d, _p, _d, _d, _d, C.c_int, _p]
        L.orc_tree_set_quadrupole.restype = C.c_int
        L.orc_tree_set_quadrupole.argtypes = [_p, C.c_int]
        L.orc_tree_nodes_q.restype = None
        L.orc_tree_nodes_q.argtypes = [_p, _p]
        L.orc_key.restype = C.c_uint64
        L.orc_key.argtypes = [_d, _d, _d, _d]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def g_p3m(R: float) -> float:
    """Cutoff function g_P3M(R) of eq. (2)."""
    return lib().orc_g_p3m(float(R))


def pair(xi, xj, m, L, r_cut, eps):
    """Acceleration at xi from a particle of mass m at xj (eq. 1, Plummer softened)."""
    out = np.zeros(3)
    lib().orc_pair(_ptr(_f64(xi)), _ptr(_f64(xj)), m, L, r_cut, eps, _ptr(out))
    return out


def _direct(fn, x, y, z, m, L, r_cut, eps, nthreads):
    x, y, z, m = map(_f64, (x, y, z, m))
    n = x.size
    ax, ay, az = np.zeros(n), np.zeros(n), np.zeros(n)
    rc = fn(n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), L, r_cut, eps, _ptr(ax), _ptr(ay), _ptr(az),
            nthreads)
    if rc != 0:
        raise ValueError(f"oracle direct sum failed ({rc})")
    return ax, ay, az


def direct_brute(x, y, z, m, L, r_cut, eps, nthreads=0):
    """Exact short-range force, all pairs (O(N^2)), minimum image."""
    return _direct(lib().orc_direct_brute, x, y, z, m, L, r_cut, eps, nthreads)


def direct_cells(x, y, z, m, L, r_cut, eps, nthreads=0):
    """Exact short-range force through a cell list (needs floor(L/r_cut) >= 3)."""
    return _direct(lib().orc_direct_cells, x, y, z, m, L, r_cut, eps, nthreads)


def theta_r(r: float, eta: float, theta0: float, theta_max: float) -> float:
    """Distance-dependent opening angle of eq. (12), r in units of eta, capped."""
    return float(lib().orc_theta_r(r, eta, theta0, theta_max))


def g_p3m_derivs(R: float):
    """(g'(R), g''(R)) of eq. (2)."""
    g1, g2 = C.c_double(), C.c_double()
    lib().orc_g_p3m_derivs(R, C.byref(g1), C.byref(g2))
    return g1.value, g2.value


def cell_acc(xi, com, M, Q, L, r_cut, eps, order=2):
    """Acceleration at xi from a cell (mass M at com, second moment Q = (xx, yy, zz, xy, xz,
    yz) about com): order 1 monopole, order 2 with the quadrupole term."""
    xi, com, Q = _f64(xi), _f64(com), _f64(Q)
    out = np.zeros(3)
    lib().orc_cell_acc(_ptr(xi), _ptr(com), float(M), _ptr(Q), L, r_cut, eps, int(order),
                       _ptr(out))
    return out


def key(x, y, z, L=1.0) -> int:
    return int(lib().orc_key(x, y, z, L))


class Tree:
    """Reference tree, groups, lists and list force for one box."""

    def __init__(self, x, y, z, m, L, r_cut, eps, theta, n_leaf, n_crit, opening=0,
                 theta_max=0.0, quadrupole=False):
        """opening=1 selects the distance-dependent angle of eq. (12): theta is then theta_0
        and theta_max its upper limit."""
        self._keep = [_f64(a) for a in (x, y, z, m)]
        x, y, z, m = self._keep
        self.n = x.size
        self.h = lib().orc_tree_build(self.n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), L, r_cut, eps,
                                      theta, n_leaf, n_crit)
        if not self.h:
            raise ValueError("oracle tree build failed")
        if opening:
            self.set_opening(opening, theta_max)
        if quadrupole:
            self.set_quadrupole(True)

    def set_quadrupole(self, on=True):
        if lib().orc_tree_set_quadrupole(self.h, 1 if on else 0) != 0:
            raise ValueError("invalid quadrupole setting")

    def nodes_q(self):
        """Second moments of the nodes about their centres of mass, (n_nodes, 6)."""
        Q = np.zeros((self.n_nodes, 6))
        lib().orc_tree_nodes_q(self.h, _ptr(Q))
        return Q

    def set_opening(self, opening, theta_max=0.0):
        if lib().orc_tree_set_opening(self.h, int(opening), float(theta_max)) != 0:
            raise ValueError("invalid opening criterion")

    def set_theta(self, theta):
        """A new opening angle on the same tree and groups (earlier lists are dropped)."""
        if lib().orc_tree_set_theta(self.h, float(theta)) != 0:
            raise ValueError("invalid theta")

    def close(self):
        if self.h:
            lib().orc_tree_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_nodes(self) -> int:
        return int(lib().orc_tree_n_nodes(self.h))

    @property
    def n_groups(self) -> int:
        return int(lib().orc_tree_n_groups(self.h))

    def sorted(self):
        k = np.zeros(self.n, dtype=np.uint64)
        i = np.zeros(self.n, dtype=np.int64)
        lib().orc_tree_sorted(self.h, _ptr(k), _ptr(i))
        return k, i

    def nodes(self):
        nn = self.n_nodes
        code = np.zeros(nn, dtype=np.uint64)
        first = np.zeros(nn, dtype=np.int64)
        count = np.zeros(nn, dtype=np.int64)
        nchild = np.zeros(nn, dtype=np.int32)
        mass, cx, cy, cz = (np.zeros(nn) for _ in range(4))
        lib().orc_tree_nodes(self.h, _ptr(code), _ptr(first), _ptr(count), _ptr(nchild),
                             _ptr(mass), _ptr(cx), _ptr(cy), _ptr(cz))
        return dict(code=code, first=first, count=count, nchild=nchild, mass=mass,
                    com=np.stack([cx, cy, cz], axis=1))

    def groups(self):
        ng = self.n_groups
        code = np.zeros(ng, dtype=np.uint64)
        first = np.zeros(ng, dtype=np.int64)
        count = np.zeros(ng, dtype=np.int64)
        lo, hi, xg = (np.zeros((ng, 3)) for _ in range(3))
        lib().orc_tree_groups(self.h, _ptr(code), _ptr(first), _ptr(count), _ptr(lo), _ptr(hi),
                              _ptr(xg))
        return dict(code=code, first=first, count=count, lo=lo, hi=hi, xg=xg)

    def lists(self):
        ne = int(lib().orc_tree_n_entries(self.h))
        if ne < 0:
            raise RuntimeError("oracle walk failed")
        off = np.zeros(self.n_groups + 1, dtype=np.int64)
        isc = np.zeros(ne, dtype=np.uint8)
        val = np.zeros(ne, dtype=np.uint64)
        if lib().orc_tree_lists(self.h, _ptr(off), _ptr(isc), _ptr(val)) != 0:
            raise RuntimeError("oracle lists failed")
        return off, isc, val

    def interactions(self) -> int:
        return int(lib().orc_tree_interactions(self.h))

    def force(self, nthreads=0):
        ax, ay, az = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        if lib().orc_tree_force(self.h, _ptr(ax), _ptr(ay), _ptr(az), nthreads) != 0:
            raise RuntimeError("oracle list force failed")
        return ax, ay, az

    def force_mag(self, nthreads=0):
        """Per particle: sum over its list of |pair force|, and of the same magnitudes
        without the cutoff factor g -- the scales of rounding error in the list force."""
        mag = np.zeros(self.n)
        newt = np.zeros(self.n)
        if lib().orc_tree_force_mag(self.h, _ptr(mag), _ptr(newt), nthreads) != 0:
            raise RuntimeError("oracle list force magnitude failed")
        return mag, newt

    def error_scale(self, nthreads=0):
        """sum_j |f_ij| + sum_j m_j r/(r^2+eps^2)^1.5 per particle: the FP64 comparison scale
        (the oracle's expanded eq. (2) rounds to a few 1e-14 of the uncut magnitude)."""
        mag, newt = self.force_mag(nthreads)
        return mag + newt

    def walk_force_sample(self, stride, offset=0, nthreads=0, scales=False):
        """Walk + list force for groups offset, offset+stride, ...; returns
        (ax, ay, az, interactions, particles) with NaN for unsampled particles, and with
        scales=True also (mag, newt), the error scales of force_mag for those particles."""
        ax, ay, az = (np.full(self.n, np.nan) for _ in range(3))
        parts = np.zeros(1, dtype=np.int64)
        mag = np.full(self.n, np.nan) if scales else None
        newt = np.full(self.n, np.nan) if scales else None
        inter = lib().orc_tree_walk_force_sample(self.h, stride, offset, _ptr(ax), _ptr(ay),
                                                 _ptr(az), nthreads, _ptr(parts),
                                                 _ptr(mag) if scales else None,
                                                 _ptr(newt) if scales else None)
        if inter < 0:
            raise RuntimeError("oracle sampled walk failed")
        out = (ax, ay, az, int(inter), int(parts[0]))
        return out + (mag, newt) if scales else out
