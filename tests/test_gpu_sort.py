"""The sort of the build (Section 2.2 step 2) at sizes of hundreds to a thousand 4096-key
tiles with ragged last tiles: the device's (key, index) order must equal the order numpy
gives to Morton keys computed here from the positions (the key rule checked against the
oracle's key function on a sample).  Clustered boxes with clumps inside one cell of side
2^-11 (equal high key bits, sorted in place as runs, and repeated positions, ordered by
index), one box with a run longer than 2048 (the whole sort then falls back to all bits)."""
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


def _spread(v):
    v = v & np.uint64(0x1FFFFF)
    for sh, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                     (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        v = (v | (v << np.uint64(sh))) & np.uint64(mask)
    return v


def _morton(x, y, z, L=1.0):
    """q = min(2^21 - 1, floor(p 2^21 / L)) per axis, bits interleaved x above y above z."""
    scale = 2097152.0 / L
    q = [np.clip(np.floor(p * scale), 0, 2097151).astype(np.uint64) for p in (x, y, z)]
    return (_spread(q[0]) << np.uint64(2)) | (_spread(q[1]) << np.uint64(1)) | _spread(q[2])


def _box(n, clumps, seed):
    x, y, z, m = boxgen.nfw_box(n, max(1, n // 2000), seed)
    rng = boxgen.SplitMix64(seed + 1)
    at = 0
    for size in clumps:
        corner = np.floor(rng.uniform(3) * 2048.0) / 2048.0
        off = rng.uniform(3 * size).reshape(3, size) * (1.0 / 2048.0)
        off[:, 4::5] = off[:, 3::5][:, : off[:, 4::5].shape[1]]
        sel = slice(at, at + size)
        x[sel], y[sel], z[sel] = corner[0] + off[0], corner[1] + off[1], corner[2] + off[2]
        at += size * 7
    return x, y, z, m


def test_key_rule_equals_the_oracle(orc):
    x, y, z, _ = _box(5000, [40], 5)
    k = _morton(x, y, z)
    for i in range(0, 5000, 7):
        assert int(k[i]) == orc.key(x[i], y[i], z[i], 1.0), i


@pytest.mark.parametrize("n,clumps", [(1_000_003, [40, 300, 9]), (4_194_321, [2000, 1, 17]),
                                      (600_001, [3000]), (4097, [])])
def test_sort_order_at_size(tp, n, clumps):
    print(f"[gpu-case] sort n={n} clumps={clumps}", flush=True)
    x, y, z, m = _box(n, clumps, 77 + n % 1000)
    p = tp.treepm_params(1.0, 1.0 / 128, 3.0 / 128, 1.0 / 2560, 0.5, 10, 256, tp.TREEPM_FP64)
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, x, y, z, m)
        gk, gi = tp.treepm_export_sorted(ctx)
    finally:
        tp.treepm_destroy(ctx)
    keys = _morton(x, y, z)
    order = np.lexsort((np.arange(n), keys))
    np.testing.assert_array_equal(gi, order)
    np.testing.assert_array_equal(gk, keys[order])
