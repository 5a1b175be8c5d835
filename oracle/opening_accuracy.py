"""Accuracy against cost of the opening criteria and of quadrupole cells, from the oracle
alone.

TEST INFRASTRUCTURE: it runs the FP64 oracle only (never the HIP library).  For a named
workload it walks a stratified sample of groups (every k-th in key order) under

  * the fixed angle theta of the walk (Section 2.2 step 5), and
  * the distance-dependent angle theta(d) = min(theta_max, theta_0 / sqrt(R g(R))),
    R = d / eta, of Section 4.1 (eq. 12),
  * the fixed angle with quadrupole cells (the second-order term of Section 4.1),

and prints, per setting, the interactions of the sampled groups and the RMS and 99th
percentile of |a - a_exact| / |a_exact| over their particles, where a_exact is the exact
short-range sum (the same walk at theta = 0, which equals the direct sum).  The HIP library's
lists equal the oracle's entry for entry, so these are also its figures, up to the FP32
kernel's rounding (RMS <= 1e-6).

    python -m oracle.opening_accuracy nfw128 --stride 200
"""
from __future__ import annotations

import argparse
import time

import numpy as np

import boxgen
import oracle


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(boxgen.CONFIGS))
    ap.add_argument("--stride", type=int, default=200)
    ap.add_argument("--n-crit", type=int, default=256)
    ap.add_argument("--fixed", default="0.4,0.5,0.6")
    ap.add_argument("--theta-r", default="0.3:0.5,0.25:0.8,0.2:0.8,0.15:0.6,0.1:0.6",
                    help="theta_0:theta_max pairs")
    ap.add_argument("--quadrupole", default="0.5,0.7",
                    help="fixed angles for rows with quadrupole cells (Section 4.1)")
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    spec, (x, y, z, m) = boxgen.config_box(a.workload)
    args = (x, y, z, m, spec.L, spec.r_cut, spec.eps)
    t0 = time.time()
    E = oracle.Tree(*args, 0.0, spec.n_leaf, a.n_crit)
    ex, ey, ez, _, parts = E.walk_force_sample(a.stride, 0, a.threads)
    E.close()
    s = ~np.isnan(ex)
    exact = np.stack([ex[s], ey[s], ez[s]])
    ne = np.linalg.norm(exact, axis=0)
    nz = ne > 0
    print(f"# {spec.name}: N={spec.n}, r_cut={spec.r_cut}, eps={spec.eps}, n_crit={a.n_crit}, "
          f"groups 0 mod {a.stride}: {parts} particles (exact sum {time.time() - t0:.1f} s)")
    print("# criterion            interactions   rms_rel     p99_rel")

    def row(label, T):
        ax, ay, az, inter, _ = T.walk_force_sample(a.stride, 0, a.threads)
        T.close()
        acc = np.stack([ax[s], ay[s], az[s]])
        e = np.linalg.norm(acc - exact, axis=0)[nz] / ne[nz]
        print(f"{label:22s} {inter:13d}   {np.sqrt(np.mean(e ** 2)):.3e}   "
              f"{np.quantile(e, 0.99):.3e}", flush=True)

    for th in (float(v) for v in a.fixed.split(",") if v):
        row(f"fixed {th}", oracle.Tree(*args, th, spec.n_leaf, a.n_crit))
    for th in (float(v) for v in a.quadrupole.split(",") if v):
        row(f"quadrupole {th}", oracle.Tree(*args, th, spec.n_leaf, a.n_crit, quadrupole=True))
    for pair in (v for v in a.theta_r.split(",") if v):
        th0, tmax = (float(v) for v in pair.split(":"))
        row(f"theta(r) {th0}/{tmax}",
            oracle.Tree(*args, th0, spec.n_leaf, a.n_crit, opening=1, theta_max=tmax))


if __name__ == "__main__":
    main()
