"""GPU parity of the time-stepping calls (treepm_timestep, treepm_kick_drift) against the FP64
oracle (oracle/integrate.py).

Both calls evaluate their formulas in plain FP64 without contraction, so the shared step and
the kicked and drifted arrays must equal the oracle's bit for bit (with float or double
accelerations).  A two-body orbit stepped with the GPU's TreePM force (FP64 short-range plus
the FP32 particle mesh) must follow the oracle's orbit to 1e-6 of the separation.
"""
import math
import sys

import numpy as np
import pytest

import boxgen
from oracle import integrate as it

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


def _ctx(tp, L=1.0, n_pm=32, eps=1e-4, theta=0.0, n_leaf=2, n_crit=1, prec=None):
    mesh = L / n_pm
    p = tp.make_params(L, mesh, 3 * mesh, eps, theta, n_leaf, n_crit,
                       tp.TREEPM_FP64 if prec is None else prec)
    return tp.treepm_create(p, 0)


def _rand(n, seed):
    rng = boxgen.SplitMix64(seed)
    return rng.uniform(3 * n).reshape(n, 3)


@pytest.mark.parametrize("acc_dtype", [np.float64, np.float32])
def test_timestep_matches_oracle(tp, acc_dtype):
    _say(f"timestep acc={np.dtype(acc_dtype).name}")
    n = 100003
    v = _rand(n, 1) - 0.5
    a = ((_rand(n, 2) - 0.5) * 1e3).astype(acc_dtype)
    a[7] = 0.0          # a particle at rest in one term only
    v[11] = 0.0
    ctx = _ctx(tp)
    try:
        vd = [torch.from_numpy(np.ascontiguousarray(v[:, c])).cuda() for c in range(3)]
        ad = [torch.from_numpy(np.ascontiguousarray(a[:, c])).cuda() for c in range(3)]
        for eps, zeta in ((1e-3, 1.0), (0.02, 2.0)):
            got = tp.treepm_timestep(ctx, *vd, *ad, eps, zeta)
            want = it.timestep(v, a.astype(np.float64), eps, zeta)
            assert got == want, (got, want)
        z = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        za = [torch.zeros(n, dtype=torch.from_numpy(a[:1, 0]).dtype, device="cuda")
              for _ in range(3)]
        assert tp.treepm_timestep(ctx, *z, *za, 1e-3, 1.0) == math.inf
    finally:
        tp.treepm_destroy(ctx)


@pytest.mark.parametrize("acc_dtype", [np.float64, np.float32])
def test_kick_drift_matches_oracle(tp, acc_dtype):
    _say(f"kick-drift acc={np.dtype(acc_dtype).name}")
    n, L = 100003, 2.5
    x = _rand(n, 3) * L
    x[0] = [0.0, np.nextafter(L, 0.0), 1e-300]   # at and next to the seam
    v = (_rand(n, 4) - 0.5) * 3.0
    a = ((_rand(n, 5) - 0.5) * 10.0).astype(acc_dtype)
    ctx = _ctx(tp, L=L)
    try:
        xd = [torch.from_numpy(np.ascontiguousarray(x[:, c])).cuda() for c in range(3)]
        vd = [torch.from_numpy(np.ascontiguousarray(v[:, c])).cuda() for c in range(3)]
        ad = [torch.from_numpy(np.ascontiguousarray(a[:, c])).cuda() for c in range(3)]
        xo, vo = x, v
        for dtk, dtd in ((0.05, 0.1), (0.1, 0.1), (-0.03, 0.2)):
            tp.treepm_kick_drift(ctx, *xd, *vd, *ad, dtk, dtd)
            xo, vo = it.kick_drift(xo, vo, a.astype(np.float64), dtk, dtd, L)
        torch.cuda.synchronize()
        gx = np.stack([t.cpu().numpy() for t in xd], axis=1)
        gv = np.stack([t.cpu().numpy() for t in vd], axis=1)
        np.testing.assert_array_equal(gv, vo)
        np.testing.assert_array_equal(gx, xo)
        assert np.all((gx >= 0.0) & (gx < L))
        # host arrays are refused before any launch
        h = np.zeros(n)
        rc = tp.lib().treepm_kick_drift(ctx, n, *([h.ctypes.data] * 9), tp.TREEPM_FP64, 0.1,
                                        0.1, None)
        assert rc == -1
    finally:
        tp.treepm_destroy(ctx)


def test_two_body_orbit_on_gpu(tp, orc):
    """The orbit of the oracle's pin (separation 0.02, N_PM = 32, 200 kick-drift steps), with
    the GPU computing every force (FP64 short-range + PM) and every kick and drift."""
    _say("two-body orbit")
    L, n_pm, eps = 1.0, 32, 1e-4
    m = np.array([0.5, 0.5])
    r0 = 0.02
    c = np.array([0.5, 0.5, 0.5])
    x = np.array([c - [r0 / 2, 0, 0], c + [r0 / 2, 0, 0]])
    ctx = _ctx(tp, L=L, n_pm=n_pm, eps=eps)
    md = torch.from_numpy(m).cuda()
    xd = [torch.from_numpy(np.ascontiguousarray(x[:, k])).cuda() for k in range(3)]
    vd = [torch.zeros(2, dtype=torch.float64, device="cuda") for _ in range(3)]
    ad = [torch.zeros(2, dtype=torch.float64, device="cuda") for _ in range(3)]

    def force():
        tp.treepm_build(ctx, *xd, md)
        tp.treepm_walk(ctx)
        tp.treepm_force_short(ctx, *ad)
        tp.treepm_force_long(ctx, *ad, accumulate=True)

    try:
        force()
        torch.cuda.synchronize()
        a0 = ad[0].cpu().numpy()
        ao = it.treepm_acc(orc, x, m, L, n_pm, eps, 0.0, n_leaf=2, n_crit=1)
        assert a0[0] == pytest.approx(ao[0, 0], rel=1e-5)
        vc = math.sqrt(ao[0, 0] * r0 / 2)
        vd[1].copy_(torch.tensor([-vc, vc], dtype=torch.float64))
        v = np.array([[0.0, -vc, 0.0], [0.0, vc, 0.0]])
        dt = 2 * math.pi * (r0 / 2) / vc / 200
        a, xo, dtk = ao, x.copy(), 0.5 * dt
        for _ in range(200):
            tp.treepm_kick_drift(ctx, *xd, *vd, *ad, dtk, dt)
            force()
            xo, v = it.kick_drift(xo, v, a, dtk, dt, L)
            a = it.treepm_acc(orc, xo, m, L, n_pm, eps, 0.0, n_leaf=2, n_crit=1)
            dtk = dt
        torch.cuda.synchronize()
        gx = np.stack([t.cpu().numpy() for t in xd], axis=1)
    finally:
        tp.treepm_destroy(ctx)
    err = np.abs(gx - xo).max()
    _say(f"  max |x_gpu - x_oracle| / r0 = {err / r0:.2e}")
    assert err <= 1e-6 * r0
    assert abs(np.linalg.norm(gx[1] - gx[0]) / r0 - 1.0) < 1e-2


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_kick_short_is_the_force_then_the_kick(tp, prec):
    """treepm_kick_short (the kick fused with the short-range force, Section 2.2 step 5) leaves
    v + dt a in the velocity arrays, bit for bit, with a the acceleration of
    treepm_force_short on the same walk; quadrupole boxes and host arrays are refused."""
    _say(f"kick_short {prec}")
    n = 20000
    x, y, z, m = boxgen.nfw_box(n, 50, 31)
    r_cut = 0.06
    precision = tp.TREEPM_FP32 if prec == "fp32" else tp.TREEPM_FP64
    p = tp.make_params(1.0, r_cut / 3, r_cut, r_cut / 60, 0.5, 10, 64, precision)
    ctx = tp.treepm_create(p, 0)
    try:
        dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
        tp.treepm_build(ctx, *dev)
        tp.treepm_walk(ctx)
        acc = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        tp.treepm_force_short(ctx, *acc)
        v0 = _rand(n, 7) - 0.5
        vel = [torch.from_numpy(np.ascontiguousarray(v0[:, c])).cuda() for c in range(3)]
        dt = 3.7e-3
        tp.treepm_kick_short(ctx, *vel, dt)
        torch.cuda.synchronize()
        a = np.stack([t.cpu().numpy() for t in acc], axis=1)
        got = np.stack([t.cpu().numpy() for t in vel], axis=1)
        ref = v0 + dt * a
        np.testing.assert_array_equal(got, ref)
        assert np.abs(a).max() > 0
        with pytest.raises(ValueError):
            tp.treepm_kick_short(ctx, *[t.cpu() for t in vel], dt)
    finally:
        tp.treepm_destroy(ctx)
    pq = tp.make_params(1.0, r_cut / 3, r_cut, r_cut / 60, 0.5, 10, 64, precision, quadrupole=1)
    ctx = tp.treepm_create(pq, 0)
    try:
        tp.treepm_build(ctx, *dev)
        tp.treepm_walk(ctx)
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_kick_short(ctx, *vel, dt)
        assert e.value.code == -1
    finally:
        tp.treepm_destroy(ctx)
