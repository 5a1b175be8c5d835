"""Kick-drift time stepping with the shared time step and softening schedule of Section 2.4 --
TEST INFRASTRUCTURE ONLY.

  * eq. (6): the softening for redshift z is eps_fin (1 + z_crit) / (1 + z) for z >= z_crit and
    eps_fin below.  Reading: this is the physical softening, so the comoving one,
    eps(z) (1 + z), is constant before z_crit and the physical one after, as the text says;
  * eq. (7): the shared step is zeta min_i(sqrt(eps / |a_i|), eps / |v_i|) (a term whose
    denominator is zero does not bind);
  * one step, as in Section 2.2 (velocities kicked by the forces, then positions drifted):
        v <- v + a dt_kick,   x <- x + v dt_drift,
    and x wrapped back into [0, L) by one box length (a value that rounds to L is 0).  The
    caller chooses dt_kick (half a step to start a leapfrog, the mean of two consecutive steps
    afterwards) and dt_drift.

Plain FP64 numpy in the order written.  The forces come from the oracle's tree and PM code.
"""
from __future__ import annotations

import numpy as np


def eps_of_z(z, eps_fin, z_crit):
    """Physical Plummer softening of eq. (6) at redshift z."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= z_crit, (1.0 + z_crit) / (1.0 + z) * eps_fin, eps_fin)


def timestep(v, a, eps, zeta):
    """eq. (7) for velocities v and accelerations a of shape (n, 3)."""
    v = np.asarray(v, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    am = np.sqrt(a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1] + a[:, 2] * a[:, 2])
    vm = np.sqrt(v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1] + v[:, 2] * v[:, 2])
    with np.errstate(divide="ignore"):
        t_a = np.where(am > 0.0, np.sqrt(eps / np.where(am > 0.0, am, 1.0)), np.inf)
        t_v = np.where(vm > 0.0, eps / np.where(vm > 0.0, vm, 1.0), np.inf)
    return zeta * min(float(t_a.min()), float(t_v.min()))


def kick_drift(x, v, a, dt_kick, dt_drift, L):
    """One kick and one drift (new arrays): v + a dt_kick, then x + v dt_drift wrapped."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64) + np.asarray(a, dtype=np.float64) * dt_kick
    xn = x + v * dt_drift
    xn = np.where(xn >= L, xn - L, xn)
    xn = np.where(xn < 0.0, xn + L, xn)
    # a coordinate just below 0 can round to L when L is added: it is at the origin
    xn = np.where(xn >= L, 0.0, xn)
    return xn, v


def treepm_acc(orc, x, m, L, n_pm, eps, theta, n_leaf=10, n_crit=64, pm_mod=None):
    """Total TreePM acceleration (tree short-range + PM long-range) from the oracle."""
    from . import pm as pm_mod_default
    pmm = pm_mod or pm_mod_default
    r_cut = 3.0 * L / n_pm
    T = orc.Tree(np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1]),
                 np.ascontiguousarray(x[:, 2]), m, L, r_cut, eps, theta, n_leaf, n_crit)
    a = np.stack(T.force(), axis=1)
    T.close()
    return a + pmm.pm_force(x, m, L, n_pm, 0.5 * r_cut)
