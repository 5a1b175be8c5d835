"""FP64 particle-mesh (PM) long-range force -- TEST INFRASTRUCTURE ONLY.

The long-range half of the TreePM split (Section 2.1; Section 2.2 step 1): mass assignment
onto an N_PM^3 mesh with the TSC (triangular shaped cloud) scheme, the potential by FFT with
the Green's function of the long-range part, and the force interpolated back to the
particles.  The paper names the steps but not the details; the readings taken here:

  * mesh points at x = i h, h = L / N_PM; a particle's TSC cloud covers the nearest mesh
    point i0 = floor(x/h + 1/2) and its two neighbours with weights
    (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2,  d = x/h - i0, per axis (periodic);
  * the potential of the mesh mass M_i is phi = (1/L^3) sum_{k != 0} G(k) M^(k) e^{i k x}
    with G(k) = phi_long^(k) / W(k)^2: phi_long^ is the Fourier transform of the long-range
    potential of a unit mass (oracle.ewald.LongRangeKernel, by quadrature of eq. (2) -- the
    complement of the cutoff function), and W(k) = prod_a sinc(k_a h / 2)^3 is the TSC
    window, divided out once for the assignment and once for the interpolation (no
    aliasing sums);
  * the mesh force is the fourth-order central difference
        F_a(i) = -[ (2/3)(phi(i+1) - phi(i-1)) - (1/12)(phi(i+2) - phi(i-2)) ] / h,
    and each particle takes the TSC-weighted sum of the 27 mesh forces around it (the same
    cloud as the assignment, so the scheme conserves momentum).

Everything is FP64 with numpy's FFT as the transform primitive.  Forces point toward the
sources, G = 1.
"""
from __future__ import annotations

import math

import numpy as np

from .ewald import LongRangeKernel


def tsc_cloud(u):
    """For coordinates u = x/h (any shape): nearest mesh index i0 and the three weights of
    the points i0-1, i0, i0+1 (last axis)."""
    u = np.asarray(u, dtype=np.float64)
    i0 = np.floor(u + 0.5)
    d = u - i0
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=-1)
    return i0.astype(np.int64), w


def assign(pos, m, L, n_pm):
    """Mesh masses M[ix, iy, iz] (sum of m_j times the product of the three axis weights)."""
    pos = np.asarray(pos, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    h = L / n_pm
    i0, w = tsc_cloud(pos / h)                     # (n, 3), (n, 3, 3)
    M = np.zeros(n_pm ** 3)
    for a in range(3):
        ix = (i0[:, 0] + a - 1) % n_pm
        for b in range(3):
            iy = (i0[:, 1] + b - 1) % n_pm
            row = (ix * n_pm + iy) * n_pm
            mw = m * w[:, 0, a] * w[:, 1, b]
            cells = np.concatenate([row + (i0[:, 2] + c - 1) % n_pm for c in range(3)])
            wts = np.concatenate([mw * w[:, 2, c] for c in range(3)])
            M += np.bincount(cells, weights=wts, minlength=n_pm ** 3)
    return M.reshape(n_pm, n_pm, n_pm)


def wavenumbers(n_pm, L):
    """k along one axis in FFT order: 2 pi n / L, n = 0 .. N/2, -N/2+1 .. -1."""
    return 2.0 * math.pi / L * np.fft.fftfreq(n_pm, d=1.0 / n_pm)


def green(n_pm, L, eta, kernel=None):
    """G(k) = phi_long^(|k|) / W(k)^2 on the mesh's wavevectors, G(0) = 0."""
    kern = kernel or LongRangeKernel(eta)
    k1 = wavenumbers(n_pm, L)
    h = L / n_pm
    s = np.ones_like(k1)
    nz = k1 != 0.0
    s[nz] = np.sin(0.5 * k1[nz] * h) / (0.5 * k1[nz] * h)
    w1 = s ** 3
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    W = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    G = np.zeros_like(kk)
    pos = kk > 0.0
    uniq, inv = np.unique(kk[pos], return_inverse=True)
    G[pos] = kern.phi_hat(uniq)[inv] / (W[pos] ** 2)
    return G


def potential(M, L, G):
    """Mesh potential: (1/L^3) sum_k G(k) M^(k) e^{ikx}, M^(k) = sum_i M_i e^{-ikx_i}."""
    n = M.shape[0]
    return np.real(np.fft.ifftn(np.fft.fftn(M) * G)) * (n ** 3) / L ** 3


def mesh_force(phi, L):
    """Fourth-order central difference of -grad phi, one array per axis."""
    h = L / phi.shape[0]
    out = []
    for a in range(3):
        p1, m1 = np.roll(phi, -1, axis=a), np.roll(phi, 1, axis=a)
        p2, m2 = np.roll(phi, -2, axis=a), np.roll(phi, 2, axis=a)
        out.append(-((2.0 / 3.0) * (p1 - m1) - (1.0 / 12.0) * (p2 - m2)) / h)
    return out


def interpolate(F, pos, L):
    """TSC-weighted sum of the mesh forces around each particle, (n, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    n_pm = F[0].shape[0]
    h = L / n_pm
    i0, w = tsc_cloud(pos / h)
    out = np.zeros((pos.shape[0], 3))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                ix = (i0[:, 0] + a - 1) % n_pm
                iy = (i0[:, 1] + b - 1) % n_pm
                iz = (i0[:, 2] + c - 1) % n_pm
                wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                for d in range(3):
                    out[:, d] += wt * F[d][ix, iy, iz]
    return out


def pm_force(pos, m, L, n_pm, eta, kernel=None, G=None):
    """Long-range PM acceleration of every particle, (n, 3)."""
    M = assign(pos, m, L, n_pm)
    if G is None:
        G = green(n_pm, L, eta, kernel)
    return interpolate(mesh_force(potential(M, L, G), L), pos, L)
