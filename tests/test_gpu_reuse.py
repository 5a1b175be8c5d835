"""Device memory kept from destroyed contexts: a context whose buffers come back from earlier
contexts (other boxes, other precisions, other parameters, so the blocks hold their values)
gives bit for bit the short- and long-range accelerations, interaction counts and lists of
the same box in a context built on freshly allocated memory; emptying the kept memory is
allowed at any time between calls and rejects devices that do not exist."""
import numpy as np
import pytest

import boxgen

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0910_0121_amd as t
    t.lib()
    return t


def _run(tp, arr, mesh, prec, n_crit=128):
    n = len(arr[0])
    p = tp.treepm_params(1.0, mesh, 3 * mesh, mesh / 20, 0.5, 10, n_crit, prec)
    dt = np.float64 if prec == tp.TREEPM_FP64 else np.float32
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, *arr)
        tp.treepm_walk(ctx)
        a = [np.zeros(n, dtype=dt) for _ in range(3)]
        tp.treepm_force_short(ctx, *a)
        b = [np.zeros(n, dtype=dt) for _ in range(3)]
        tp.treepm_force_long(ctx, *b)
        st = tp.treepm_get_stats(ctx)
        off, isc, val = tp.treepm_export_lists(ctx)
        return np.stack(a), np.stack(b), st.interactions, off, isc, val
    finally:
        tp.treepm_destroy(ctx)


def _same(r, s):
    for u, v in zip(r, s):
        if isinstance(u, np.ndarray):
            np.testing.assert_array_equal(u, v)
        else:
            assert u == v


def test_reused_buffers_give_the_results_of_fresh_ones(tp):
    print("[gpu-case] reuse of kept device memory", flush=True)
    box = boxgen.nfw_box(150_001, 75, 61)
    other = boxgen.nfw_box(260_000, 130, 62)
    small = boxgen.uniform_box(20_000, 63)
    mesh = 1.0 / 32
    tp.treepm_release_cached(0)
    fresh32 = _run(tp, box, mesh, tp.TREEPM_FP32)
    tp.treepm_release_cached(0)
    fresh64 = _run(tp, box, mesh, tp.TREEPM_FP64)
    for k in range(3):
        # leave blocks of other sizes and contents behind, then run the box on them
        _run(tp, other, 1.0 / 64, tp.TREEPM_FP64 if k % 2 else tp.TREEPM_FP32, 64 + 96 * k)
        _run(tp, small, 1.0 / 16, tp.TREEPM_FP32, 32)
        _same(_run(tp, box, mesh, tp.TREEPM_FP32), fresh32)
        _same(_run(tp, box, mesh, tp.TREEPM_FP64), fresh64)


def test_release_cached_between_calls_and_bad_devices(tp):
    box = boxgen.uniform_box(30_000, 64)
    mesh = 1.0 / 16
    p = tp.treepm_params(1.0, mesh, 3 * mesh, mesh / 20, 0.5, 10, 64, tp.TREEPM_FP32)
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, *box)
        tp.treepm_release_cached(0)  # the live context keeps its buffers
        tp.treepm_walk(ctx)
        a = [np.zeros(30_000, dtype=np.float32) for _ in range(3)]
        tp.treepm_force_short(ctx, *a)
    finally:
        tp.treepm_destroy(ctx)
    tp.treepm_release_cached(0)
    tp.treepm_release_cached(0)
    ref = _run(tp, box, mesh, tp.TREEPM_FP32, 64)
    np.testing.assert_array_equal(np.stack(a), ref[0])
    for bad in (-1, torch.cuda.device_count(), 1 << 20):
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_release_cached(bad)
        assert e.value.code == -4
