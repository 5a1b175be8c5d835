"""Pins of the oracle's pair law and exact short-range sums against what the paper and the
mathematics fix (no GPU).

* eq. (2) (Section 2.1): exact values, C^3 joins at R = 1, flatness at R = 2, the factored
  branch-2 form, the Newtonian limit, and -- independently of the printed coefficients --
  1 - g(R) equals the mass within r = R*eta of the self-convolution of two S2 clouds of
  radius eta (the Hockney & Eastwood shape the paper cites for g_P3M).
* eq. (1) with Plummer softening (Section 2.4): two-body closed form across the periodic
  boundary, zero at and beyond r_cut, Newton's third law, a perfect lattice feels no force,
  translation invariance, and two independent pair enumerations agree.
* The TreePM split (Section 2.1; Section 3.1.2 uses an Ewald sum as the exact force): short
  (minimum image, eq. 1) + Fourier long-range part = Ewald periodic force, with the Ewald sum
  itself pinned by independence of its splitting parameter and by symmetry.
"""
import math

import numpy as np
import pytest
from scipy.special import roots_legendre

import boxgen


# ----------------------------------------------------------------------------- eq. (2)

def test_g_exact_values(orc):
    assert orc.g_p3m(0.0) == 1.0
    assert orc.g_p3m(1.0) == pytest.approx(43.0 / 140.0, rel=0, abs=1e-15)
    assert orc.g_p3m(2.0) == 0.0
    assert orc.g_p3m(2.5) == 0.0
    assert orc.g_p3m(100.0) == 0.0


def _deriv(f, x, side, order, h):
    """One-sided finite differences (side = -1 uses points below x, +1 above)."""
    pts = [f(x + side * k * h) for k in range(order + 4)]
    if order == 1:   # 4th-order one-sided first derivative
        c = [-25 / 12, 4, -3, 4 / 3, -1 / 4]
        return side * sum(ci * p for ci, p in zip(c, pts)) / h
    if order == 2:
        c = [15 / 4, -77 / 6, 107 / 6, -13, 61 / 12, -5 / 6]
        return sum(ci * p for ci, p in zip(c, pts)) / h ** 2
    if order == 3:
        c = [-49 / 8, 29, -461 / 8, 62, -307 / 8, 13, -15 / 8]
        return side * sum(ci * p for ci, p in zip(c, pts)) / h ** 3
    raise ValueError


@pytest.mark.parametrize("order,expect,h,tol", [(1, -1.0, 1e-3, 1e-8),
                                                (2, 7.0 / 5.0, 1e-2, 1e-5),
                                                (3, 24.0 / 5.0, 2e-2, 2e-3)])
def test_g_joins_c3_at_one(orc, order, expect, h, tol):
    """Both branches of eq. (2) meet at R = 1 with equal 1st, 2nd and 3rd derivatives."""
    below = _deriv(orc.g_p3m, 1.0 - 1e-15, -1, order, h)
    above = _deriv(orc.g_p3m, 1.0, +1, order, h)
    assert below == pytest.approx(expect, abs=tol)
    assert above == pytest.approx(expect, abs=tol)


def test_g_flat_at_two(orc):
    """Branch 2 vanishes to 5th order at R = 2: g(2-h)/h^5 -> 168/140.  (h stays where g is
    well above the ~1e-14 rounding of the expanded polynomial.)"""
    for h in (5e-2, 1e-2):
        assert orc.g_p3m(2.0 - h) / h ** 5 == pytest.approx(168.0 / 140.0, rel=2 * h)


def test_g_branch2_factored(orc):
    """Branch 2 of eq. (2) equals (2-R)^5 (7R^3 + 22R^2 + 10R + 4) / 140.  The printed,
    expanded form cancels terms of size ~30 on [1, 2), so it carries ~1e-14 absolute rounding."""
    for R in np.linspace(1.0, 1.999, 37):
        f = (2.0 - R) ** 5 * (7 * R ** 3 + 22 * R ** 2 + 10 * R + 4) / 140.0
        assert orc.g_p3m(R) == pytest.approx(f, rel=0, abs=3e-14)


def test_g_newtonian_limit(orc):
    """Well inside r_cut the pair law is Newtonian: 1 - g(R) = (8/5) R^3 + O(R^5)."""
    for R in (1e-2, 3e-3, 1e-3):
        assert (1.0 - orc.g_p3m(R)) / R ** 3 == pytest.approx(1.6, rel=2 * R * R + 1e-9)


def _gl(a, b, n):
    x, w = roots_legendre(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _s2_pair_mass_within(r, a=1.0):
    """Mass within radius r of rho*rho, rho = S2 cloud of radius a (density falling linearly
    to zero at a, unit mass), by nested Gauss-Legendre quadrature split at every kink."""
    rho = lambda t: np.where(t < a, 3.0 / (math.pi * a ** 3) * (1.0 - t / a), 0.0)

    def conv(s):  # radial self-convolution (rho*rho)(s)
        tot = 0.0
        brk = sorted({0.0, a} | {v for v in (s, a - s, s - a) if 0.0 < v < a})
        for lo, hi in zip(brk[:-1], brk[1:]):
            rr, ww = _gl(lo, hi, 24)
            for ri, wi in zip(rr, ww):
                t0, t1 = abs(s - ri), min(s + ri, a)
                if t1 > t0:
                    tt, tw = _gl(t0, t1, 12)
                    tot += wi * ri * rho(ri) * np.sum(tw * tt * rho(tt))
        return 2.0 * math.pi / s * tot

    tot = 0.0
    for lo, hi in ((0.0, min(r, a)), (min(r, a), r)):
        if hi > lo:
            s, w = _gl(lo, hi, 24)
            tot += sum(wi * 4.0 * math.pi * si * si * conv(si) for si, wi in zip(s, w))
    return tot


@pytest.mark.parametrize("R", [0.25, 0.6, 0.95, 1.0, 1.35, 1.8, 2.0])
def test_g_is_s2_cloud_complement(orc, R):
    """g_P3M is the Hockney-Eastwood S2 split: 1 - g(r/eta) is the fraction of the force of
    two S2 clouds of radius eta that has not been cut, i.e. the mass of their
    self-convolution within r.  Fixes every coefficient of eq. (2) independently."""
    assert 1.0 - orc.g_p3m(R) == pytest.approx(_s2_pair_mass_within(R), abs=1e-12)


# ----------------------------------------------------------------------------- eq. (1)

def test_two_body_across_boundary(orc):
    """Two particles straddling the x boundary: closed form m d g(|d|/eta)/(|d|^2+eps^2)^1.5,
    pointing from each particle to the other's nearest image."""
    L, r_cut, eps = 1.0, 0.2, 1e-3
    x = np.array([0.02, 0.98]); y = np.array([0.5, 0.53]); z = np.array([0.5, 0.49])
    m = np.array([0.3, 0.7])
    ax, ay, az = orc.direct_brute(x, y, z, m, L, r_cut, eps)
    d = np.array([-0.04, 0.03, -0.01])  # particle 1 minus particle 0, nearest image
    r = np.linalg.norm(d)
    f = orc.g_p3m(r / (0.5 * r_cut)) / (r * r + eps * eps) ** 1.5
    np.testing.assert_allclose([ax[0], ay[0], az[0]], m[1] * f * d, rtol=1e-12)
    np.testing.assert_allclose([ax[1], ay[1], az[1]], -m[0] * f * d, rtol=1e-12)


def test_zero_at_and_beyond_cutoff(orc):
    L, r_cut, eps = 1.0, 0.1, 1e-3
    for sep, expect_zero in ((0.1, True), (0.1000001, True), (0.3, True), (0.0999, False)):
        x = np.array([0.3, 0.3 + sep]); y = np.full(2, 0.5); z = np.full(2, 0.5)
        ax, _, _ = orc.direct_brute(x, y, z, np.ones(2), L, r_cut, eps)
        assert (ax[0] == 0.0) == expect_zero, sep
        assert ax[0] >= 0.0  # attraction toward the source (+x)


def test_pair_newtonian_well_inside_cutoff(orc):
    """|a| r^2 / m = 1 - (8/5)(r/eta)^3 + ... for eps << r << eta (here r/eta = 1e-3)."""
    a = orc.pair([0.5, 0.5, 0.5], [0.5 + 1e-4, 0.5, 0.5], 2.0, 1.0, 0.2, 0.0)
    assert a[0] * 1e-8 / 2.0 == pytest.approx(1.0 - 1.6e-9, rel=1e-11)


def _box(n, seed):
    return boxgen.uniform_box(n, seed)


def test_net_force_vanishes(orc):
    x, y, z, m = _box(3000, 5)
    ax, ay, az = orc.direct_brute(x, y, z, m, 1.0, 0.12, 0.004)
    net = np.array([np.sum(m * ax), np.sum(m * ay), np.sum(m * az)])
    scale = np.sum(m * np.sqrt(ax * ax + ay * ay + az * az))
    assert np.all(np.abs(net) <= 1e-13 * scale)


def test_perfect_lattice_feels_no_force(orc):
    k = 8
    g = (np.arange(k) + 0.5) / k
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    m = np.full(x.size, 1.0 / x.size)
    r_cut, eps = 3.0 / k, 0.01
    ax, ay, az = orc.direct_brute(x, y, z, m, 1.0, r_cut, eps)
    # scale: one nearest-neighbour pair force
    f1 = np.linalg.norm(orc.pair([0.5, 0.5, 0.5], [0.5 + 1.0 / k, 0.5, 0.5], m[0], 1.0, r_cut,
                                 eps))
    assert np.max(np.abs(np.concatenate([ax, ay, az]))) <= 1e-12 * f1


def test_translation_invariance(orc):
    x, y, z, m = _box(2000, 6)
    a0 = np.stack(orc.direct_brute(x, y, z, m, 1.0, 0.15, 0.005))
    s = np.array([0.3711, 0.9123, 0.0457])
    xs, ys, zs = ((p + d) % 1.0 for p, d in zip((x, y, z), s))
    a1 = np.stack(orc.direct_brute(xs, ys, zs, m, 1.0, 0.15, 0.005))
    scale = np.max(np.linalg.norm(a0, axis=0))
    assert np.max(np.abs(a1 - a0)) <= 1e-11 * scale


@pytest.mark.parametrize("seed,n,r_cut", [(7, 4000, 0.1), (8, 2500, 0.25)])
def test_brute_equals_cell_list(orc, seed, n, r_cut):
    x, y, z, m = _box(n, seed)
    a = np.stack(orc.direct_brute(x, y, z, m, 1.0, r_cut, r_cut / 60))
    b = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, r_cut / 60))
    scale = np.max(np.linalg.norm(a, axis=0))
    assert np.max(np.abs(a - b)) <= 1e-13 * scale


# ----------------------------------------------------------------------------- split

def _tiny(n=16, seed=11):
    x, y, z, m = boxgen.uniform_box(n, seed)
    return np.stack([x, y, z], axis=1), m


def test_ewald_alpha_independent():
    from oracle import ewald
    pos, m = _tiny()
    F5 = ewald.ewald_force(pos, m, 1.0, 5.0)
    F7 = ewald.ewald_force(pos, m, 1.0, 7.0, nmax_k=20)
    assert np.max(np.abs(F5 - F7)) <= 1e-12 * np.max(np.abs(F5))


def test_ewald_symmetric_pair_is_force_free():
    from oracle import ewald
    pos = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]])
    F = ewald.ewald_force(pos, np.ones(2), 1.0, 5.0)
    assert np.max(np.abs(F)) < 1e-12


def test_ewald_newtonian_at_short_range():
    from oracle import ewald
    d = 1e-3
    pos = np.array([[0.4, 0.5, 0.5], [0.4 + d, 0.5, 0.5]])
    F = ewald.ewald_force(pos, np.ones(2), 1.0, 5.0)
    assert F[0, 0] * d * d == pytest.approx(1.0, abs=1e-7)
    assert F[1, 0] == pytest.approx(-F[0, 0], rel=1e-12)


def test_short_plus_long_is_periodic_force(orc):
    """F_short (eq. 1, minimum image, eps = 0) + F_long = F_Ewald.  The Fourier sum for F_long
    is truncated at |n_a| <= nmax; its error falls as the cut grows (roughly nmax^-4 here),
    so the check demands both a small residual and that it shrinks."""
    from oracle import ewald
    pos, m = _tiny()
    L, r_cut = 1.0, 0.45
    ax, ay, az = orc.direct_brute(pos[:, 0], pos[:, 1], pos[:, 2], m, L, r_cut, 0.0)
    Fs = np.stack([ax, ay, az], axis=1)
    Fe = ewald.ewald_force(pos, m, L, 5.0)
    ker = ewald.LongRangeKernel(0.5 * r_cut)
    err = {}
    for nmax in (16, 32):
        Fl = ewald.long_range_force(pos, m, L, 0.5 * r_cut, nmax=nmax, kernel=ker)
        err[nmax] = np.max(np.abs(Fs + Fl - Fe)) / np.max(np.abs(Fe))
    assert err[32] < 2e-8
    assert err[32] < err[16] / 5.0
    # The long-range kernel tends to the Newtonian -4 pi / k^2 at long wavelength.
    k = np.array([1e-2])
    assert ker.phi_hat(k)[0] * k[0] ** 2 / (-4 * math.pi) == pytest.approx(1.0, abs=1e-5)
