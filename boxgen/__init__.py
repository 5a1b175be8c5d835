"""Seeded synthetic particle boxes shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and places particles.  It holds none of the
tree-force arithmetic, so the oracle and the HIP path can both take their inputs from it
without sharing any of the method's code.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used as a counter-based generator: output number k of a
stream with seed s is mix(s + k * 0x9E3779B97F4A7C15) for k = 1, 2, ...  A uniform double
in [0, 1) is (z >> 11) * 2**-53.

Boxes stand in for the paper's LCDM snapshots (Section 3, generated with GRAFIC, which are
not available): a uniform box, and a clustered box of NFW halos (concentration 10, halo
masses drawn from dN/dM ~ M^-1.9 over two decades, truncated at r_200) plus a uniform
background.  Every particle has mass 1/N, the box is the unit cube (Section 3.1.1 normalises
the box to unity).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "SplitMix64",
    "uniform_box",
    "nfw_box",
    "config_box",
    "serving_sizes",
    "CONFIGS",
    "BoxSpec",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


_CHUNK = 1 << 18


def _mix(z: np.ndarray) -> np.ndarray:
    # numpy's uint64 array-times-scalar loop is very slow on some builds; multiplying by a
    # full array of the constant takes the fast elementwise path.
    n = z.size
    s30, s27, s31 = (np.full(1, v, dtype=np.uint64) for v in (30, 27, 31))
    z = (z ^ (z >> s30)) * _const(_M1, n)
    z = (z ^ (z >> s27)) * _const(_M2, n)
    return z ^ (z >> s31)


_CONST_CACHE: dict = {}


def _const(v, n):
    key = (int(v), n)
    a = _CONST_CACHE.get(key)
    if a is None:
        a = np.full(n, v, dtype=np.uint64)
        if n == _CHUNK:
            _CONST_CACHE[key] = a
    return a


class SplitMix64:
    """Counter-based SplitMix64 stream; ``next_u64(n)`` returns the next n outputs."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.counter = 0

    def next_u64(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.uint64)
        # Work in cache-sized chunks so no large temporaries are created.
        with np.errstate(over="ignore"):
            for s in range(0, n, _CHUNK):
                c = min(_CHUNK, n - s)
                k = np.arange(self.counter + 1 + s, self.counter + 1 + s + c, dtype=np.uint64)
                out[s:s + c] = _mix(_const(self.seed, c) + k * _const(_GOLDEN, c))
        self.counter += n
        return out

    def uniform(self, n: int) -> np.ndarray:
        """n doubles in [0, 1) with 53 random bits each."""
        out = np.empty(n, dtype=np.float64)
        sh = np.full(1, 11, dtype=np.uint64)
        for s in range(0, n, _CHUNK):
            c = min(_CHUNK, n - s)
            out[s:s + c] = (self.next_u64(c) >> sh).astype(np.float64) * (2.0 ** -53)
        return out


def _wrap_unit(v: np.ndarray, L: float) -> np.ndarray:
    """Map into [0, L) in place: v - L*floor(v/L), a result equal to L becomes 0."""
    for s in range(0, v.size, _CHUNK):
        w = v[s:s + _CHUNK]
        w -= L * np.floor(w / L)
        w[(w >= L) | (w < 0.0)] = 0.0
    return v


def uniform_box(n: int, seed: int, L: float = 1.0):
    """n particles uniform i.i.d. in [0, L)^3, mass 1/n; x block, then y, then z from one stream."""
    rng = SplitMix64(seed)
    x = rng.uniform(n) * L
    y = rng.uniform(n) * L
    z = rng.uniform(n) * L
    # u * L < L for L = 1; guard other L against rounding up to L.
    for a in (x, y, z):
        a[a >= L] = 0.0
    m = np.full(n, 1.0 / n)
    return x, y, z, m


def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def _nfw_radius_units(u: np.ndarray, c: float = 10.0) -> np.ndarray:
    """Solve mu(x)/mu(c) = u for x in [0, c] (mu(x) = ln(1+x) - x/(1+x)).

    Bracketed Newton iteration: the bracket [lo, hi] always holds the root, a Newton step that
    leaves it is replaced by bisection, and an element stops once its step falls below
    2^-50 of its value (a few FP64 ulps).  Each element's iteration depends on that element
    alone, so the variates are solved in cache-sized chunks.
    """
    out = np.empty_like(u)
    for s in range(0, u.size, _CHUNK):
        out[s:s + _CHUNK] = _nfw_radius_chunk(u[s:s + _CHUNK], c)
    return out


def _nfw_radius_chunk(u: np.ndarray, c: float) -> np.ndarray:
    target = u * _nfw_mu(np.float64(c))
    lo = np.zeros_like(u)
    hi = np.full_like(u, c)
    x = np.full_like(u, 1.0)
    idx = np.arange(u.size)
    for _ in range(200):
        if idx.size == 0:
            break
        xa = x[idx]
        f = _nfw_mu(xa) - target[idx]
        below = f < 0
        la = np.where(below, xa, lo[idx])
        ha = np.where(below, hi[idx], xa)
        lo[idx] = la
        hi[idx] = ha
        d = xa / ((1.0 + xa) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = xa - f / d
        bad = ~((xn >= la) & (xn <= ha)) | ~np.isfinite(xn)
        xn = np.where(bad, 0.5 * (la + ha), xn)
        conv = (np.abs(xn - xa) <= 2.0 ** -50 * np.maximum(xa, 1e-300)) | (f == 0)
        x[idx] = xn
        idx = idx[~conv]
    return x


def _stable_argsort_u64(k: np.ndarray) -> np.ndarray:
    """The stable argsort of k.  Without repeated values every sort gives the same order, so
    the faster unstable sort is used and the stable one only if two values are equal."""
    perm = np.argsort(k)
    ks = k[perm]
    if np.any(ks[1:] == ks[:-1]):
        perm = np.argsort(k, kind="stable")
    return perm


def nfw_box(n: int, n_halos: int, seed: int, f_halo: float = 0.5, L: float = 1.0,
            concentration: float = 10.0):
    """Clustered box: a fraction f_halo of the n particles in n_halos NFW halos, the rest uniform.

    Draw order from one SplitMix64 stream: halo masses (n_halos), halo centres (x block,
    y block, z block), then for all halo particles in halo order: radius variates, cos(polar)
    variates, azimuth variates; then the uniform remainder (x, y, z blocks); then one 64-bit
    key per particle whose stable argsort gives the final random order.
    """
    rng = SplitMix64(seed)
    # Halo masses from dN/dM ~ M^-1.9 on [1, 100] by inverse CDF.
    u = rng.uniform(n_halos)
    mh = (1.0 - u * (1.0 - 100.0 ** -0.9)) ** (-1.0 / 0.9)
    cx = rng.uniform(n_halos) * L
    cy = rng.uniform(n_halos) * L
    cz = rng.uniform(n_halos) * L
    # Particle counts proportional to halo mass, largest-remainder rounding.
    n_in = int(round(f_halo * n))
    share = mh / mh.sum() * n_in
    cnt = np.floor(share).astype(np.int64)
    rem = n_in - int(cnt.sum())
    if rem > 0:
        order = np.argsort(-(share - cnt), kind="stable")
        cnt[order[:rem]] += 1
    n_h = int(cnt.sum())
    # Radii: r_200 from the halo's mass fraction at mean density 1 (unit box, total mass 1).
    m_frac = cnt.astype(np.float64) / n
    r200 = (3.0 * m_frac * L ** 3 / (800.0 * math.pi)) ** (1.0 / 3.0)
    rs = r200 / concentration
    halo_of = np.repeat(np.arange(n_halos), cnt)
    ur = rng.uniform(n_h)
    xr = _nfw_radius_units(ur, concentration)
    r = xr * rs[halo_of]
    r = np.minimum(r, r200[halo_of])
    ct = 2.0 * rng.uniform(n_h) - 1.0
    ph = 2.0 * math.pi * rng.uniform(n_h)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    hx = cx[halo_of] + r * st * np.cos(ph)
    hy = cy[halo_of] + r * st * np.sin(ph)
    hz = cz[halo_of] + r * ct
    n_u = n - n_h
    ux = rng.uniform(n_u) * L
    uy = rng.uniform(n_u) * L
    uz = rng.uniform(n_u) * L
    x = _wrap_unit(np.concatenate([hx, ux]), L)
    y = _wrap_unit(np.concatenate([hy, uy]), L)
    z = _wrap_unit(np.concatenate([hz, uz]), L)
    perm = _stable_argsort_u64(rng.next_u64(n))
    m = np.full(n, 1.0 / n)
    return (np.ascontiguousarray(x[perm]), np.ascontiguousarray(y[perm]),
            np.ascontiguousarray(z[perm]), m)


@dataclass(frozen=True)
class BoxSpec:
    """One workload: box contents plus the tree-force parameters used on it."""
    name: str
    n: int
    kind: str          # "uniform" | "nfw"
    n_halos: int
    f_halo: float
    seed: int
    mesh_n: int        # PM mesh points per side; mesh spacing = L / mesh_n
    theta: float
    n_crit: int
    n_leaf: int = 10
    L: float = 1.0

    @property
    def mesh(self) -> float:
        return self.L / self.mesh_n

    @property
    def r_cut(self) -> float:
        # Section 2.2, step 1: 2 eta = r_cut = 3 / N_PM (box normalised to 1).
        return 3.0 * self.mesh

    @property
    def eps(self) -> float:
        return self.mesh / 20.0

    def generate(self):
        if self.kind == "uniform":
            return uniform_box(self.n, self.seed, self.L)
        return nfw_box(self.n, self.n_halos, self.seed, self.f_halo, self.L)


CONFIGS = {
    "uniform32k": BoxSpec("uniform32k", 32 ** 3, "uniform", 0, 0.0, 1, 32, 0.5, 64),
    "nfw128": BoxSpec("nfw128", 128 ** 3, "nfw", 200, 0.5, 2, 128, 0.5, 128),
    "nfw256": BoxSpec("nfw256", 256 ** 3, "nfw", 2000, 0.5, 3, 256, 0.5, 128),
    "nfw512": BoxSpec("nfw512", 512 ** 3, "nfw", 10000, 0.7, 4, 512, 0.5, 128),
}


def config_box(name: str):
    spec = CONFIGS[name]
    return spec, spec.generate()


def serving_sizes(n_boxes: int = 64, seed: int = 999):
    """Box sizes log-uniform in [32^3, 256^3] and halo counts max(1, round(N/1e4))."""
    rng = SplitMix64(seed)
    u = rng.uniform(n_boxes)
    lo, hi = math.log(32 ** 3), math.log(256 ** 3)
    ns = np.rint(np.exp(lo + u * (hi - lo))).astype(np.int64)
    halos = np.maximum(1, np.rint(ns / 1.0e4)).astype(np.int64)
    return ns, halos
