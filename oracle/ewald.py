"""Periodic Ewald sum and the Fourier long-range (PM-like) force -- TEST INFRASTRUCTURE ONLY.

These pin the cutoff function g_P3M of eq. (2) (Section 2.1) as the exact complement of the
long-range part of the TreePM split: for a tiny periodic box with no softening,

    F_short (minimum image, eq. 1, all pairs closer than r_cut)  +  F_long  =  F_Ewald,

where F_Ewald is the exact periodic Newtonian force (Section 3.1.2 measures the total force
error against a direct Ewald summation) and F_long is the Fourier series of what the cutoff
function removes.  Everything is FP64; the k = 0 mode is dropped in both sums (uniform
neutralising background).  G = 1; forces point toward the sources.

Long-range potential of a unit mass: phi_long(r) = -1/r + psi(r), with
    psi(r) = 1/r - 1/(2 eta) - int_r^{2 eta} (1 - g(s/eta)) / s^2 ds      (r < 2 eta, else 0)
the negative of the short-range potential whose gradient is the pair law of eq. (1).  Its
Fourier transform is
    phi_long^(k) = -4 pi / k^2 + (4 pi / k) int_0^{2 eta} r psi(r) sin(k r) dr,
evaluated here by Gauss-Legendre quadrature of the g of eq. (2); no closed-form shape factor
is used.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, roots_legendre


def g_p3m_vec(R):
    """Eq. (2) on an array (same formula as the C oracle, for quadrature)."""
    R = np.asarray(R, dtype=np.float64)
    R2, R3 = R * R, R * R * R
    R4, R5, R6, R7, R8 = R3 * R, R3 * R2, R3 * R3, R3 * R3 * R, R3 * R3 * R2
    b1 = 1.0 - (224.0 * R3 - 224.0 * R5 + 70.0 * R6 + 48.0 * R7 - 21.0 * R8) / 140.0
    b2 = 1.0 - (12.0 - 224.0 * R2 + 896.0 * R3 - 840.0 * R4 + 224.0 * R5 + 70.0 * R6
                - 48.0 * R7 + 7.0 * R8) / 140.0
    return np.where(R < 1.0, b1, np.where(R < 2.0, b2, 0.0))


def _gl(a, b, n):
    x, w = roots_legendre(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _inner(r, eta, n=48):
    """int_r^{2 eta} (1 - g(s/eta)) / s^2 ds for each r in [0, 2 eta], split at s = eta
    (where eq. (2) changes branch) so each piece has a smooth integrand."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    for k, rk in enumerate(r):
        tot = 0.0
        pieces = [(rk, eta), (eta, 2.0 * eta)] if rk < eta else [(rk, 2.0 * eta)]
        for a, b in pieces:
            if b <= a:
                continue
            s, w = _gl(a, b, n)
            tot += np.sum(w * (1.0 - g_p3m_vec(s / eta)) / (s * s))
        out[k] = tot
    return out


class LongRangeKernel:
    """phi_long^(k) for the cutoff of eq. (2) with scale eta, by quadrature."""

    def __init__(self, eta: float, n_outer: int = 160):
        self.eta = eta
        # Outer nodes on [0, eta] and [eta, 2 eta]; r psi(r) tabulated once.
        r1, w1 = _gl(0.0, eta, n_outer)
        r2, w2 = _gl(eta, 2.0 * eta, n_outer)
        self.r = np.concatenate([r1, r2])
        self.w = np.concatenate([w1, w2])
        inner = _inner(self.r, eta)
        self.rpsi = 1.0 - self.r / (2.0 * eta) - self.r * inner

    def phi_hat(self, k):
        k = np.asarray(k, dtype=np.float64)
        integ = np.sin(np.multiply.outer(k, self.r)) @ (self.w * self.rpsi)
        return -4.0 * math.pi / (k * k) + 4.0 * math.pi / k * integ


def _kvectors(nmax: int, L: float):
    rng = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), axis=-1).reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    return n, (2.0 * math.pi / L) * n.astype(np.float64)


def _sin_sum(kv, pos, m):
    """For each particle i and k: sum_j m_j sin(k.(x_i - x_j)) = Im(e^{i k.x_i} S(k)),
    S(k) = sum_j m_j e^{-i k.x_j}.  Shape (n_k, n)."""
    ph = kv @ pos.T                      # (n_k, n)
    S = (m[None, :] * np.exp(-1j * ph)).sum(axis=1)
    return np.imag(np.exp(1j * ph) * S[:, None])


def long_range_force(pos, m, L, eta, nmax=24, kernel=None):
    """F_long,i = (1/L^3) sum_{k != 0} phi_long^(k) k sum_j m_j sin(k.(x_i - x_j))."""
    pos = np.asarray(pos, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    kern = kernel or LongRangeKernel(eta)
    n_int, kv = _kvectors(nmax, L)
    n2 = (n_int * n_int).sum(axis=1)
    uniq, inv = np.unique(n2, return_inverse=True)
    kmag = (2.0 * math.pi / L) * np.sqrt(uniq.astype(np.float64))
    ph = kern.phi_hat(kmag)[inv]          # (n_k,)
    ss = _sin_sum(kv, pos, m)             # (n_k, n)
    return (kv[:, None, :] * (ph[:, None] * ss)[:, :, None]).sum(axis=0) / L ** 3


def ewald_force(pos, m, L, alpha, n_real=2, nmax_k=16):
    """Exact periodic Newtonian force (k = 0 dropped), Ewald split with Gaussian width 1/alpha.

    Real space: sum over images |n_a| <= n_real of
        m_j [erfc(alpha r)/r^2 + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)/r] r_vec/r,
        r_vec = x_j - x_i + n L, excluding j = i with n = 0;
    Fourier space: (4 pi/L^3) sum_{k != 0} m_j (k/k^2) exp(-k^2/(4 alpha^2)) sin(k.(x_j - x_i)).
    """
    pos = np.asarray(pos, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    n = pos.shape[0]
    F = np.zeros((n, 3))
    rng = np.arange(-n_real, n_real + 1)
    img = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), axis=-1).reshape(-1, 3) * L
    for i in range(n):
        rv = (pos[None, :, :] - pos[i][None, None, :]) + img[:, None, :]   # (n_img, n, 3)
        r = np.sqrt((rv * rv).sum(axis=-1))
        mask = r > 0.0
        rs = np.where(mask, r, 1.0)
        mag = (erfc(alpha * rs) / (rs * rs)
               + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * rs) ** 2) / rs)
        mag = np.where(mask, mag * m[None, :], 0.0)
        F[i] = ((mag / rs)[:, :, None] * rv).sum(axis=(0, 1))
    _, kv = _kvectors(nmax_k, L)
    k2 = (kv * kv).sum(axis=1)
    coef = 4.0 * math.pi / L ** 3 * np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    ss = _sin_sum(kv, pos, m)             # sum_j m_j sin(k.(x_i - x_j))
    F += -(kv[:, None, :] * (coef[:, None] * ss)[:, :, None]).sum(axis=0)
    return F
