"""Parity at the scale workload: the 512^3 clustered box (10,000 NFW halos holding 70 % of the
particles, mesh 512^3, r_cut = 3/512, eps = 1/(20*512)) at theta = 0.4 and 0.5 (Table 2 of the
paper runs a 512^3 box at theta = 0.5; Section 3.2 follows how the interactions grow as theta
falls), n_crit = 192, the group size the benchmark's 512^3 leg runs.

The box is built, walked and forced on the GPU in FP64 and FP32.  The oracle builds the whole
tree once and, for each theta, walks and sums the lists of every 4000th group in key order;
the GPU's forces on those groups' particles are checked with the bars of the other full-size
tests (FP64: 1e-13 of the summed magnitudes per particle and component; FP32: RMS relative
error <= 1e-6 and none above 2e-4).  The interaction totals of the two GPU paths agree, and
more interactions are needed at theta = 0.4 than at 0.5.

Generating the box and building the oracle's tree take a minute or two each on the host;
progress lines are written as each step ends.
"""
import sys
import time

import numpy as np
import pytest

import boxgen

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N_CRIT = 192
STRIDE = 4000


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0910_0121_amd as t
    t.lib()
    return t


@pytest.fixture(scope="module")
def say(pytestconfig):
    capman = pytestconfig.pluginmanager.getplugin("capturemanager")

    def _say(msg):
        # straight to the terminal, so a long host step is followed by a line at its end
        with capman.global_and_fixture_disabled():
            print(f"[gpu-case] {msg}", flush=True)
        sys.stdout.flush()
    return _say


@pytest.fixture(scope="module")
def box512(say):
    t0 = time.time()
    spec, arrays = boxgen.config_box("nfw512")
    say(f"nfw512: generated N={spec.n} in {time.time() - t0:.0f} s")
    return spec, arrays


@pytest.fixture(scope="module")
def oracle512(orc, box512, say):
    spec, (x, y, z, m) = box512
    t0 = time.time()
    T = orc.Tree(x, y, z, m, spec.L, spec.r_cut, spec.eps, 0.5, spec.n_leaf, N_CRIT)
    say(f"nfw512: oracle tree {T.n_nodes} nodes, {T.n_groups} groups in "
        f"{time.time() - t0:.0f} s")
    yield T
    T.close()


def _gpu(tp, spec, dev, theta, precision):
    p = tp.make_params(spec.L, spec.mesh, spec.r_cut, spec.eps, theta, spec.n_leaf, N_CRIT,
                       precision)
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, *dev)
        st = tp.treepm_walk(ctx)
        acc = [torch.zeros(spec.n, dtype=torch.float64, device="cuda") for _ in range(3)]
        tp.treepm_force_short(ctx, *acc)
        torch.cuda.synchronize()
        return [a.cpu().numpy() for a in acc], st
    finally:
        tp.treepm_destroy(ctx)


_INTER = {}


@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_scale512_sampled_parity(tp, box512, oracle512, say, theta):
    spec, arrays = box512
    T = oracle512
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    a64, st64 = _gpu(tp, spec, dev, theta, tp.TREEPM_FP64)
    say(f"theta={theta}: FP64 path done ({st64.interactions} interactions, "
        f"{st64.n_groups} groups)")
    a32, st32 = _gpu(tp, spec, dev, theta, tp.TREEPM_FP32)
    del dev
    torch.cuda.empty_cache()
    say(f"theta={theta}: FP32 path done")
    assert st64.interactions == st32.interactions
    assert st64.n_groups == T.n_groups and st64.n_nodes == T.n_nodes
    _INTER[theta] = st64.interactions
    T.set_theta(theta)
    t0 = time.time()
    ax, ay, az, inter, parts, mag, newt = T.walk_force_sample(STRIDE, 0, 16, scales=True)
    say(f"theta={theta}: oracle sample {parts} particles, {inter} interactions in "
        f"{time.time() - t0:.0f} s")
    s = ~np.isnan(ax)
    assert s.sum() == parts > 10000
    ref = np.stack([ax[s], ay[s], az[s]])
    scale = (mag + newt)[s]
    err64 = np.abs(np.stack([a[s] for a in a64]) - ref)
    say(f"  fp64 max |da|/scale {np.max(err64 / scale):.2e}")
    assert np.all(err64 <= 1e-13 * scale[None, :])
    d = np.linalg.norm(np.stack([a[s] for a in a32]) - ref, axis=0)
    nr = np.linalg.norm(ref, axis=0)
    nz = nr > 0
    rel = d[nz] / nr[nz]
    rms = float(np.sqrt(np.mean(rel ** 2)))
    say(f"  fp32 rms rel {rms:.3e} max rel {rel.max():.3e} p99 {np.quantile(rel, 0.99):.3e}")
    assert rms <= 1e-6 and rel.max() <= 2e-4
    assert np.all(d[~nz] == 0.0)
    if 0.5 in _INTER and 0.4 in _INTER:
        assert _INTER[0.4] > _INTER[0.5]
