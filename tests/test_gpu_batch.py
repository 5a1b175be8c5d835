"""Shared launches (treepm_force_short_batch): the walk and FP32 short-range force of several
boxes in one traversal launch and one force launch per size class give, for every box, exactly
the accelerations and counts of treepm_walk + treepm_force_short on that box alone.  Covers
boxes walked before (one-pass lists sized from their last walk) beside fresh ones (two passes),
different N, opening rules and quadrupole cells, boxes of a few hundred particles, device outputs,
a box whose one-pass pool is too small (walked again alone inside the call), and the argument
checks."""
import ctypes as C

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


def _create(tp, prm):
    """A context whose later walks use the one-pass pool whatever the box size (these boxes
    are below the size where the automatic choice takes it)."""
    ctx = tp.treepm_create(prm, 0)
    tp.treepm_set_walk_passes(ctx, tp.TREEPM_WALK_ONE_PASS)
    return ctx


def _params(tp, mesh, theta=0.5, opening=0, theta_max=0.0, quad=0, n_crit=128, L=1.0):
    return tp.make_params(L, mesh, 3 * mesh, mesh / 20, theta, 10, n_crit, tp.TREEPM_FP32,
                          opening=opening, theta_max=theta_max, quadrupole=quad)


def _cases(tp):
    """(params, arrays) of boxes with different sizes, clustering and modes."""
    out = []
    for kind, n, seed, extra in [("nfw", 60000, 41, {}), ("uniform", 30011, 42, {}),
                                 ("nfw", 90000, 43, dict(theta=0.3, opening=1, theta_max=0.5)),
                                 ("nfw", 45000, 44, dict(quad=1)),
                                 ("uniform", 100, 45, dict(n_crit=16)),
                                 ("uniform", 700, 46, dict(n_crit=8)),
                                 ("nfw", 20000, 47, dict(n_crit=32))]:
        arr = boxgen.uniform_box(n, seed) if kind == "uniform" else boxgen.nfw_box(n, max(1, n // 500), seed)
        # (the FP32 path needs every group's cube half-side + r_cut <= L/2: tiny boxes get a
        # fine mesh and small groups)
        mesh_n = max(16, round(n ** (1 / 3)))
        out.append((_params(tp, 1.0 / mesh_n, **extra), arr))
    return out


def _alone(tp, prm, arr):
    ctx = tp.treepm_create(prm, 0)
    try:
        tp.treepm_build(ctx, *arr)
        tp.treepm_walk(ctx)
        a = [np.zeros(len(arr[0]), dtype=np.float32) for _ in range(3)]
        tp.treepm_force_short(ctx, *a)
        st = tp.treepm_get_stats(ctx)
        return np.stack(a), (st.interactions, st.n_cell_entries, st.n_part_entries, st.evaluated)
    finally:
        tp.treepm_destroy(ctx)


def _counts(tp, ctx):
    st = tp.treepm_get_stats(ctx)
    return (st.interactions, st.n_cell_entries, st.n_part_entries, st.evaluated)


def test_batch_equals_alone(tp):
    print("[gpu-case] batch of 7 boxes vs each alone, fresh then walked", flush=True)
    cases = _cases(tp)
    ref = [_alone(tp, prm, arr) for prm, arr in cases]
    ctxs = [_create(tp, prm) for prm, _ in cases]
    try:
        # boxes 1 and 3 walked before: their lists go into pools sized from that walk
        for k in (1, 3):
            tp.treepm_build(ctxs[k], *cases[k][1])
            tp.treepm_walk(ctxs[k])
        for rep in range(2):
            for c, (prm, arr) in zip(ctxs, cases):
                tp.treepm_build(c, *arr)
            outs = [tuple(np.full(len(arr[0]), np.nan, dtype=np.float32) for _ in range(3))
                    for _, arr in cases]
            tp.treepm_force_short_batch(ctxs, outs)
            for b, (c, o) in enumerate(zip(ctxs, outs)):
                np.testing.assert_array_equal(np.stack(o), ref[b][0], err_msg=f"box {b} rep {rep}")
                assert _counts(tp, c) == ref[b][1], (b, rep)
            # the single-box force after a batch walk gives the same again
            a = [np.zeros(len(cases[0][1][0]), dtype=np.float32) for _ in range(3)]
            tp.treepm_force_short(ctxs[0], *a)
            np.testing.assert_array_equal(np.stack(a), ref[0][0])
    finally:
        for c in ctxs:
            tp.treepm_destroy(c)


def test_batch_n_crit_256_and_distinct_tables(tp):
    """Groups of up to 256 particles (every blocking factor K = 1..4 of the force classes) and
    boxes whose pair-law tables differ (eps / r_cut of 1/20, 1/30 and 1/40: the force
    launch reloads the table between boxes), each equal to its alone result."""
    print("[gpu-case] batch with n_crit 256 and three pair-law tables", flush=True)
    cases = []
    for n, seed, eps_div in [(120000, 71, 20), (50000, 72, 40), (200000, 73, 30),
                             (80000, 74, 20), (30000, 75, 40)]:
        arr = boxgen.nfw_box(n, max(1, n // 500), seed)
        mesh = 1.0 / round(n ** (1 / 3))
        prm = tp.make_params(1.0, mesh, 3 * mesh, 3 * mesh / eps_div, 0.5, 10, 256,
                             tp.TREEPM_FP32)
        cases.append((prm, arr))
    ref = [_alone(tp, prm, arr) for prm, arr in cases]
    ctxs = [_create(tp, prm) for prm, _ in cases]
    try:
        for rep in range(2):
            for c, (prm, arr) in zip(ctxs, cases):
                tp.treepm_build(c, *arr)
            outs = [tuple(np.full(len(arr[0]), np.nan, dtype=np.float32) for _ in range(3))
                    for _, arr in cases]
            tp.treepm_force_short_batch(ctxs, outs)
            for b, (c, o) in enumerate(zip(ctxs, outs)):
                np.testing.assert_array_equal(np.stack(o), ref[b][0], err_msg=f"box {b} rep {rep}")
                assert _counts(tp, c) == ref[b][1], (b, rep)
    finally:
        for c in ctxs:
            tp.treepm_destroy(c)


def test_batch_large_boxes(tp):
    """Boxes of 0.3 to 4 million particles (up to 8 groups per XCD part of every class and
    tens of thousands of groups per box), mixed with a small one, equal to their alone
    results; then again with all of them walked before (one-pass pools)."""
    print("[gpu-case] batch of large boxes", flush=True)
    cases = []
    for n, seed in [(4_000_000, 81), (300_000, 82), (1_500_000, 83), (20_000, 84)]:
        arr = boxgen.nfw_box(n, max(1, n // 5000), seed)
        mesh = 1.0 / round(n ** (1 / 3))
        cases.append((tp.make_params(1.0, mesh, 3 * mesh, mesh / 20, 0.5, 10, 256,
                                     tp.TREEPM_FP32), arr))
    ref = [_alone(tp, prm, arr) for prm, arr in cases]
    ctxs = [_create(tp, prm) for prm, _ in cases]
    try:
        for rep in range(2):
            for c, (prm, arr) in zip(ctxs, cases):
                tp.treepm_build(c, *arr)
            outs = [tuple(np.full(len(arr[0]), np.nan, dtype=np.float32) for _ in range(3))
                    for _, arr in cases]
            tp.treepm_force_short_batch(ctxs, outs)
            for b, (c, o) in enumerate(zip(ctxs, outs)):
                np.testing.assert_array_equal(np.stack(o), ref[b][0], err_msg=f"box {b} rep {rep}")
                assert _counts(tp, c) == ref[b][1], (b, rep)
    finally:
        for c in ctxs:
            tp.treepm_destroy(c)


def test_batch_device_outputs_and_one_box(tp):
    print("[gpu-case] batch with device outputs; batch of one", flush=True)
    cases = _cases(tp)[:3]
    ref = [_alone(tp, prm, arr) for prm, arr in cases]
    ctxs = [_create(tp, prm) for prm, _ in cases]
    try:
        for c, (prm, arr) in zip(ctxs, cases):
            tp.treepm_build(c, *arr)
        outs = [tuple(torch.empty(len(arr[0]), dtype=torch.float32, device="cuda")
                      for _ in range(3)) for _, arr in cases]
        tp.treepm_force_short_batch(ctxs, outs)
        torch.cuda.synchronize()
        for b, o in enumerate(outs):
            np.testing.assert_array_equal(torch.stack(o).cpu().numpy(), ref[b][0])
        tp.treepm_build(ctxs[2], *cases[2][1])
        o = tuple(np.zeros(len(cases[2][1][0]), dtype=np.float32) for _ in range(3))
        tp.treepm_force_short_batch([ctxs[2]], [o])
        np.testing.assert_array_equal(np.stack(o), ref[2][0])
    finally:
        for c in ctxs:
            tp.treepm_destroy(c)


def test_batch_pool_too_small_walks_again(tp):
    """A context last walked on a small box sizes a pool whose chunks are shorter than the
    lists of the large box it now holds (theta = 0, r_cut = 0.3 L): its lists are walked again
    in two passes inside the call, and every box still equals its alone result."""
    print("[gpu-case] batch with a one-pass pool that is too small", flush=True)
    prm = _params(tp, 0.1, theta=0.0, n_crit=64)
    small = boxgen.uniform_box(2000, 51)
    big = boxgen.uniform_box(150000, 52)
    other_prm, other = _params(tp, 1.0 / 40), boxgen.nfw_box(64000, 128, 53)
    ref_big, ref_other = _alone(tp, prm, big), _alone(tp, other_prm, other)
    c_big, c_other = _create(tp, prm), _create(tp, other_prm)
    try:
        tp.treepm_build(c_big, *small)
        tp.treepm_walk(c_big)
        tp.treepm_build(c_big, *big)
        tp.treepm_build(c_other, *other)
        tp.treepm_walk(c_other)
        tp.treepm_build(c_other, *other)
        o_big = tuple(np.zeros(len(big[0]), dtype=np.float32) for _ in range(3))
        o_other = tuple(np.zeros(len(other[0]), dtype=np.float32) for _ in range(3))
        tp.treepm_force_short_batch([c_other, c_big], [o_other, o_big])
        np.testing.assert_array_equal(np.stack(o_big), ref_big[0])
        np.testing.assert_array_equal(np.stack(o_other), ref_other[0])
        assert _counts(tp, c_big) == ref_big[1]
        assert _counts(tp, c_other) == ref_other[1]
    finally:
        tp.treepm_destroy(c_big)
        tp.treepm_destroy(c_other)


def test_batch_argument_checks(tp):
    print("[gpu-case] batch argument checks", flush=True)
    lib = tp.lib()
    x, y, z, m = boxgen.uniform_box(3000, 61)
    p32 = _params(tp, 1.0 / 14)
    p64 = tp.make_params(1.0, 1.0 / 14, 3.0 / 14, 1.0 / 280, 0.5, 10, 64, tp.TREEPM_FP64)
    a, b, c64 = tp.treepm_create(p32, 0), tp.treepm_create(p32, 0), tp.treepm_create(p64, 0)
    try:
        o = tuple(np.zeros(3000, dtype=np.float32) for _ in range(3))
        with pytest.raises(tp.TreePMError) as e:  # not built
            tp.treepm_force_short_batch([a], [o])
        assert e.value.code == -5
        tp.treepm_build(a, x, y, z, m)
        tp.treepm_build(b, x, y, z, m)
        tp.treepm_build(c64, x, y, z, m)
        with pytest.raises(tp.TreePMError) as e:  # FP64 box
            tp.treepm_force_short_batch([a, c64], [o, o])
        assert e.value.code == -1 and "FP32" in str(e.value)
        with pytest.raises(tp.TreePMError) as e:  # a box twice
            tp.treepm_force_short_batch([a, b, a], [o, o, o])
        assert e.value.code == -1
        arr = C.c_void_p * 17
        none = arr()
        assert lib.treepm_force_short_batch(arr(*([a] * 17)), 17, none, none, none,
                                            tp.TREEPM_HOST, None) == -1
        assert lib.treepm_force_short_batch(arr(a), 0, none, none, none, tp.TREEPM_HOST,
                                            None) == -1
        # the checks left both boxes built: a batch of the two still works
        ref = _alone(tp, p32, (x, y, z, m))
        o2 = tuple(np.zeros(3000, dtype=np.float32) for _ in range(3))
        tp.treepm_force_short_batch([a, b], [o, o2])
        np.testing.assert_array_equal(np.stack(o), ref[0])
        np.testing.assert_array_equal(np.stack(o2), ref[0])
    finally:
        for h in (a, b, c64):
            tp.treepm_destroy(h)
