"""GPU parity of the particle-mesh long-range force (treepm_force_long) against the FP64 oracle
(oracle/pm.py) on the same seeded boxes.

The mesh arithmetic is FP32 (assignment sums are exact in fixed point; the FFT, Green's
function, differences and interpolation round in FP32), so the bar is relative to the force
scale of the box: RMS over particles of |a_gpu - a_oracle| at most 2e-6 of the RMS |a_oracle|,
and no particle above 5e-5 of it.  A radix-2 FFT in FP32 keeps the rounding of each mesh value
near log2(N_PM) u of the mesh's RMS (u = 2^-24, log2 N <= 8 here), the differences and the
27-point interpolation add a few u, and the Green's table is rounded once.  The results must
also be bit-for-bit repeatable (the fixed-point mass sums do not depend on the order of the
atomics).
"""
import sys

import numpy as np
import pytest

import boxgen
from oracle import pm

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0910_0121_amd as t
    t.lib()
    return t


def _long(tp, x, y, z, m, n_pm, L=1.0, dtype=torch.float64, host=False, accumulate_onto=None):
    mesh = L / n_pm
    p = tp.make_params(L, mesh, 3.0 * mesh, mesh / 20.0, 0.5, 10, 64, tp.TREEPM_FP32)
    ctx = tp.treepm_create(p, 0)
    try:
        dev = "cpu" if host else "cuda"
        tp.treepm_build(ctx, *[torch.from_numpy(np.ascontiguousarray(a)).cuda()
                               for a in (x, y, z, m)])
        if accumulate_onto is None:
            out = [torch.zeros(len(x), dtype=dtype, device=dev) for _ in range(3)]
            tp.treepm_force_long(ctx, *out)
        else:
            out = [torch.from_numpy(a.copy()).to(dev) for a in accumulate_onto]
            tp.treepm_force_long(ctx, *out, accumulate=True)
        torch.cuda.synchronize()
        return np.stack([t.cpu().numpy().astype(np.float64) for t in out], axis=1)
    finally:
        tp.treepm_destroy(ctx)


def _check(got, ref, what):
    scale = float(np.sqrt(np.mean((ref * ref).sum(axis=1))))
    d = np.linalg.norm(got - ref, axis=1)
    rms = float(np.sqrt(np.mean(d * d))) / scale
    mx = float(d.max()) / scale
    _say(f"  {what}: rms |da| / rms |a| = {rms:.2e}, max {mx:.2e}")
    assert rms <= 2e-6 and mx <= 5e-5


CASES = [
    # kind, n, seed, n_pm
    ("uniform", 32768, 1, 32),     # the plain-method box (32^3 particles, 32^3 mesh)
    ("nfw", 40000, 2, 64),
    ("nfw", 20011, 3, 16),         # ragged N, the smallest mesh
    ("uniform", 5000, 4, 128),     # more mesh points than particles
]


def test_pm_unequal_masses(tp):
    """Masses spread over more than three decades, the heaviest particle last in the caller's
    order: the fixed-point scale of the assignment comes from the largest mass, which the
    build reduces over many blocks while it permutes the records.  A scale taken from the
    wrong maximum would overflow the 64-bit sums or lose their precision."""
    _say("pm unequal masses")
    n = 100003
    x, y, z, _ = boxgen.nfw_box(n, 200, 7)
    m = np.exp(boxgen.SplitMix64(8).uniform(n) * np.log(1e3))
    m[-1] = 5e3
    m /= m.sum()
    got = _long(tp, x, y, z, m, 64)
    ref = pm.pm_force(np.stack([x, y, z], axis=1), m, 1.0, 64, 1.5 / 64)
    _check(got, ref, "unequal masses")


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-n{c[1]}-pm{c[3]}" for c in CASES])
def test_pm_force_matches_oracle(tp, case):
    kind, n, seed, n_pm = case
    _say(f"pm {kind} n={n} N_PM={n_pm}")
    if kind == "uniform":
        x, y, z, m = boxgen.uniform_box(n, seed)
    else:
        x, y, z, m = boxgen.nfw_box(n, max(1, n // 400), seed)
    got = _long(tp, x, y, z, m, n_pm)
    ref = pm.pm_force(np.stack([x, y, z], axis=1), m, 1.0, n_pm, 1.5 / n_pm)
    _check(got, ref, "fp64 out")
    again = _long(tp, x, y, z, m, n_pm)
    np.testing.assert_array_equal(got, again)
    got32 = _long(tp, x, y, z, m, n_pm, dtype=torch.float32)
    np.testing.assert_array_equal(got32, got.astype(np.float32).astype(np.float64))


def test_pm_particles_on_the_seams(tp):
    """Clouds that wrap around the periodic boundary: particles at 0, just below L and at
    half-cell offsets from the seam on every axis, among a clustered box."""
    x, y, z, m = boxgen.nfw_box(20000, 40, 6)
    L, n_pm = 1.0, 32
    h = L / n_pm
    seam = np.array([0.0, np.nextafter(L, 0.0), 0.5 * h, L - 0.5 * h, 0.25 * h, L - 0.25 * h])
    k = seam.size
    x[:k], y[:k], z[:k] = seam, seam[::-1].copy(), np.roll(seam, 2)
    got = _long(tp, x, y, z, m, n_pm)
    ref = pm.pm_force(np.stack([x, y, z], axis=1), m, L, n_pm, 1.5 * h)
    _check(got, ref, "seam particles")
    d = np.linalg.norm(got[:k] - ref[:k], axis=1)
    scale = float(np.sqrt(np.mean((ref * ref).sum(axis=1))))
    assert np.all(d <= 5e-5 * scale)


def test_pm_box_size_and_host_buffers(tp):
    """L = 2.5 with host output buffers, and accumulation onto existing values."""
    x, y, z, m = boxgen.nfw_box(30000, 60, 5)
    L = 2.5
    x, y, z = 2.5 * x, 2.5 * y, 2.5 * z
    got = _long(tp, x, y, z, m, 32, L=L, host=True)
    ref = pm.pm_force(np.stack([x, y, z], axis=1), m, L, 32, 1.5 * L / 32)
    _check(got, ref, "L = 2.5, host buffers")
    base = [np.full(len(x), 0.25), np.arange(len(x), dtype=np.float64) * 1e-3,
            np.full(len(x), -3.0)]
    acc = _long(tp, x, y, z, m, 32, L=L, accumulate_onto=base)
    np.testing.assert_allclose(acc - np.stack(base, axis=1), got, rtol=0,
                               atol=1e-12 * np.abs(got).max() + 4e-16 * 3.0)


def test_pm_total_force_is_short_plus_long(tp, orc):
    """treepm_force_short then treepm_force_long(accumulate) gives the TreePM total; with
    theta = 0 and eps = 0 on 16 particles it must reproduce the Ewald force as the oracle's
    own short + PM sum does (RMS 4.0e-3 at N_PM = 32, r_cut = 3 h)."""
    from oracle import ewald
    rng = boxgen.SplitMix64(5)
    pos = rng.uniform(48).reshape(16, 3)
    m = np.full(16, 1.0 / 16)
    x, y, z = (np.ascontiguousarray(pos[:, a]) for a in range(3))
    p = tp.make_params(1.0, 1 / 32, 3 / 32, 0.0, 0.0, 2, 4, tp.TREEPM_FP64)
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, *[torch.from_numpy(a).cuda() for a in (x, y, z, m)])
        tp.treepm_walk(ctx)
        a = [torch.zeros(16, dtype=torch.float64, device="cuda") for _ in range(3)]
        tp.treepm_force_short(ctx, *a)
        tp.treepm_force_long(ctx, *a, accumulate=True)
        torch.cuda.synchronize()
        tot = np.stack([t.cpu().numpy() for t in a], axis=1)
    finally:
        tp.treepm_destroy(ctx)
    Fe = ewald.ewald_force(pos, m, 1.0, 8.0, n_real=2, nmax_k=16)
    fs = np.stack(orc.direct_brute(x, y, z, m, 1.0, 3 / 32, 0.0), axis=1)
    ref = fs + pm.pm_force(pos, m, 1.0, 32, 1.5 / 32)
    _check(tot, ref, "short + long vs oracle")
    e = np.linalg.norm(tot - Fe, axis=1) / np.linalg.norm(Fe, axis=1)
    assert float(np.sqrt(np.mean(e ** 2))) < 6e-3


def test_pm_errors(tp):
    x, y, z, m = (torch.from_numpy(a).cuda() for a in boxgen.uniform_box(1000, 1))
    out = [torch.zeros(1000, dtype=torch.float64, device="cuda") for _ in range(3)]
    for mesh in (1 / 48, 1 / 8, 1 / 2048):      # not a power of two; too coarse; too fine
        p = tp.make_params(1.0, mesh, 3 * mesh, 0.001, 0.5, 10, 64, tp.TREEPM_FP64)
        ctx = tp.treepm_create(p, 0)
        try:
            tp.treepm_build(ctx, x, y, z, m)
            with pytest.raises(tp.TreePMError) as e:
                tp.treepm_force_long(ctx, *out)
            assert e.value.code == -1, mesh
        finally:
            tp.treepm_destroy(ctx)
    p = tp.make_params(1.0, 1 / 32, 3 / 32, 0.001, 0.5, 10, 64, tp.TREEPM_FP64)
    ctx = tp.treepm_create(p, 0)
    try:
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_force_long(ctx, *out)        # before any build
        assert e.value.code == -5
    finally:
        tp.treepm_destroy(ctx)


@pytest.mark.parametrize("n", [1, 2, 7])
def test_pm_tiny_boxes(tp, n):
    """A handful of particles (one wave's chunk partly empty, most of the mesh empty).  The
    forces can nearly vanish (one particle: only its mesh self-force), so the bar is relative
    to the mesh's own force scale M / h^2: 1e-6 of it."""
    rng = boxgen.SplitMix64(40 + n)
    pos = rng.uniform(3 * n).reshape(n, 3)
    m = np.full(n, 1.0 / n)
    x, y, z = (np.ascontiguousarray(pos[:, a]) for a in range(3))
    got = _long(tp, x, y, z, m, 16)
    ref = pm.pm_force(pos, m, 1.0, 16, 1.5 / 16)
    scale = m.sum() / (1.0 / 16) ** 2
    assert np.abs(got - ref).max() <= 1e-6 * scale
