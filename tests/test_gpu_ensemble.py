"""Ensemble serving on the GPU: several boxes submitted together give, for every request,
exactly the accelerations the same box gives alone through the single-box calls (same
kernels, same inputs, per-box state), each request run alone or with shared launches; a
tight HBM budget forces queueing and eviction without changing results; errors are reported
per request."""
import time

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


def _boxes():
    out = []
    for i, (kind, n, seed) in enumerate([("uniform", 40000, 31), ("nfw", 60000, 32),
                                         ("nfw", 30011, 33), ("nfw", 90000, 34)]):
        arr = boxgen.uniform_box(n, seed) if kind == "uniform" else boxgen.nfw_box(n, n // 500, seed)
        mesh_n = round(n ** (1 / 3))
        out.append((i, arr, 1.0 / mesh_n))
    return out


def _params(tp, mesh):
    return tp.treepm_params(1.0, mesh, 3 * mesh, mesh / 20, 0.5, 10, 128, tp.TREEPM_FP32)


def _alone(tp, arr, mesh):
    ctx = tp.treepm_create(_params(tp, mesh), 0)
    try:
        tp.treepm_build(ctx, *arr)
        tp.treepm_walk(ctx)
        a = [np.zeros(len(arr[0]), dtype=np.float32) for _ in range(3)]
        tp.treepm_force_short(ctx, *a)
        return np.stack(a), tp.treepm_get_stats(ctx).interactions
    finally:
        tp.treepm_destroy(ctx)


def _drain(tp, ens, tickets, sizes, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            n = sizes[t]
            a = [np.zeros(n, dtype=np.float32) for _ in range(3)]
            rc, st = tp.treepm_ensemble_poll(ens, t, *a)
            if rc == tp.TREEPM_OK:
                res[t] = (np.stack(a), st)
        assert time.time() - t0 < timeout, "ensemble did not finish"
        time.sleep(0.002)
    return res


@pytest.mark.parametrize("budget_boxes,inflight,batching",
                         [(100, 4, False), (1.2, 2, False), (100, 4, True), (1.2, 2, True)])
def test_mix_equals_alone(tp, budget_boxes, inflight, batching):
    print(f"[gpu-case] ensemble budget={budget_boxes} boxes inflight={inflight} "
          f"batching={batching}", flush=True)
    boxes = _boxes()
    ref = {i: _alone(tp, arr, mesh) for i, arr, mesh in boxes}
    biggest = max(len(arr[0]) for _, arr, _ in boxes)
    budget = int(budget_boxes * (biggest * 320 + (64 << 20)))
    ens = tp.treepm_ens_create(0, budget, inflight)
    if batching:
        tp.treepm_ens_set_batching(ens, True)
    try:
        tickets, sizes, which = [], {}, {}
        for rep in range(3):
            for i, arr, mesh in boxes[::-1] if rep % 2 else boxes:
                t = tp.treepm_ensemble_submit(ens, i, _params(tp, mesh), *arr)
                tickets.append(t)
                sizes[t] = len(arr[0])
                which[t] = i
        res = _drain(tp, ens, tickets, sizes)
        for t in tickets:
            a, st = res[t]
            np.testing.assert_array_equal(a, ref[which[t]][0])
            assert st.interactions == ref[which[t]][1]
            assert st.latency_ms > 0
            assert 1 <= st.batch_boxes <= (16 if batching else 1)
            assert min(st.stage_ms) >= 0 and sum(st.stage_ms) <= st.latency_ms - st.queue_ms + 1e-6
        info = tp.treepm_ens_info(ens)
        assert info["queued"] == 0 and info["inflight"] == 0
        if budget_boxes < 2:
            assert info["resident_boxes"] <= 2
    finally:
        tp.treepm_ens_destroy(ens)


@pytest.mark.parametrize("batching", [False, True])
def test_modes_mix_equals_alone(tp, batching):
    """Boxes with the distance-dependent opening angle and with quadrupole cells, served in one
    mix, give exactly what each gives alone with the same parameters."""
    print(f"[gpu-case] ensemble with opening and quadrupole modes, batching={batching}",
          flush=True)
    boxes = _boxes()

    def params(i, mesh):
        return tp.make_params(1.0, mesh, 3 * mesh, mesh / 20, 0.3 if i % 2 == 0 else 0.5, 10,
                              128, tp.TREEPM_FP32,
                              opening=tp.TREEPM_OPEN_DISTANCE if i % 2 == 0 else 0,
                              theta_max=0.5 if i % 2 == 0 else 0.0, quadrupole=i // 2)

    ref = {}
    for i, arr, mesh in boxes:
        ctx = tp.treepm_create(params(i, mesh), 0)
        try:
            tp.treepm_build(ctx, *arr)
            tp.treepm_walk(ctx)
            a = [np.zeros(len(arr[0]), dtype=np.float32) for _ in range(3)]
            tp.treepm_force_short(ctx, *a)
            ref[i] = (np.stack(a), tp.treepm_get_stats(ctx).interactions)
        finally:
            tp.treepm_destroy(ctx)
    biggest = max(len(arr[0]) for _, arr, _ in boxes)
    ens = tp.treepm_ens_create(0, int(100 * (biggest * 320 + (64 << 20))), 4)
    tp.treepm_ens_set_batching(ens, batching)
    try:
        tickets, sizes, which = [], {}, {}
        for rep in range(2):
            for i, arr, mesh in boxes:
                t = tp.treepm_ensemble_submit(ens, i, params(i, mesh), *arr)
                tickets.append(t)
                sizes[t] = len(arr[0])
                which[t] = i
        res = _drain(tp, ens, tickets, sizes)
        for t in tickets:
            a, st = res[t]
            np.testing.assert_array_equal(a, ref[which[t]][0])
            assert st.interactions == ref[which[t]][1]
    finally:
        tp.treepm_ens_destroy(ens)


def test_errors(tp):
    print("[gpu-case] ensemble errors", flush=True)
    ens = tp.treepm_ens_create(0, 256 << 20, 2)
    try:
        x, y, z, m = boxgen.uniform_box(5000, 7)
        p = _params(tp, 1.0 / 17)
        # a box that can never fit the budget is refused at submit
        big = 10 ** 6
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_ensemble_submit(ens, 9, p, np.zeros(big), np.zeros(big), np.zeros(big),
                                      np.ones(big))
        assert e.value.code == -3
        # invalid parameters
        bad = tp.treepm_params(1.0, 0.2, 0.6, 0.01, 0.5, 10, 64, tp.TREEPM_FP32)
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_ensemble_submit(ens, 1, bad, x, y, z, m)
        assert e.value.code == -1
        # a position out of range fails that request only
        xb = x.copy(); xb[3] = 1.5
        t_bad = tp.treepm_ensemble_submit(ens, 2, p, xb, y, z, m)
        t_ok = tp.treepm_ensemble_submit(ens, 3, p, x, y, z, m)
        t0 = time.time()
        while True:
            try:
                rc, _ = tp.treepm_ensemble_poll(ens, t_bad)
            except tp.TreePMError as err:
                assert err.code == -2
                break
            assert time.time() - t0 < 60
            time.sleep(0.002)
        res = _drain(tp, ens, [t_ok], {t_ok: 5000})
        np.testing.assert_array_equal(res[t_ok][0], _alone(tp, (x, y, z, m), 1.0 / 17)[0])
        # a released or unknown ticket
        with pytest.raises(tp.TreePMError):
            tp.treepm_ensemble_poll(ens, t_ok)
        with pytest.raises(tp.TreePMError):
            tp.treepm_ensemble_poll(ens, 123456789)
        # destroy with work still queued returns promptly
        for k in range(20):
            tp.treepm_ensemble_submit(ens, 100 + k, p, x, y, z, m)
    finally:
        t0 = time.time()
        tp.treepm_ens_destroy(ens)
        assert time.time() - t0 < 60
