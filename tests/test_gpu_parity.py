"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the same seeded
boxes.

Bars:
  * keys, sort order, tree nodes, node masses/centres of mass, groups and interaction lists:
    bit-identical (the walk's FP64 decisions are taken with the same IEEE operations);
  * FP64 forces: |a_gpu - a_oracle| <= 1e-13 * (sum_j |f_ij| + sum_j N_ij) per particle and
    component, N_ij = m_j r/(r^2+eps^2)^1.5 the magnitude without the cutoff factor:
    summation order differs, and the oracle's expanded eq. (2) rounds to a few 1e-14 of the
    uncut magnitude near R = 2 (its terms reach ~300 there) while the kernel's factored form
    does not;
  * FP32 forces: RMS over particles of |a_gpu - a_oracle| / |a_oracle| <= 1e-6 on the same
    lists, and per particle |da_i| <= 8 u B_i with u = 2^-24 and
    B_i = sum_j m_j (|x_i - x_g|_inf + |x_j - x_g|_inf + r_ij) / (r_ij^2 + eps^2)^1.5:
    rounding the group-relative positions to FP32 moves d by at most ~u(|x_i'| + |x_j'|), the
    pair law's Jacobian is at most 4 m / (r^2 + eps^2)^1.5, and the pair arithmetic adds a
    few u of |f_ij| <= m r / (r^2 + eps^2)^1.5.  Particles whose exact force is zero must get
    exactly zero.
"""
import os
import sys

import numpy as np
import pytest

import boxgen

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


class Run:
    def __init__(self, tp, x, y, z, m, L, r_cut, eps, theta, n_leaf, n_crit, precision,
                 out64=True, host=False):
        self.tp = tp
        p = tp.treepm_params(L, r_cut / 3.0, r_cut, eps, theta, n_leaf, n_crit, precision)
        self.ctx = tp.treepm_create(p, 0)
        dev = "cpu" if host else "cuda"
        xs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, y, z, m)]
        tp.treepm_build(self.ctx, *xs)
        self.stats = tp.treepm_walk(self.ctx)
        dt = torch.float64 if out64 else torch.float32
        self.a = [torch.zeros(len(x), dtype=dt, device=dev) for _ in range(3)]
        tp.treepm_force_short(self.ctx, *self.a)
        torch.cuda.synchronize()
        self.acc = np.stack([t.cpu().numpy().astype(np.float64) for t in self.a])

    def close(self):
        if self.ctx:
            self.tp.treepm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _box(kind, n, seed):
    if kind == "uniform":
        return boxgen.uniform_box(n, seed)
    x, y, z, m = boxgen.nfw_box(n, max(1, n // 400), seed)
    if kind == "nfw-masses":  # masses over three decades
        m = np.exp(boxgen.SplitMix64(seed + 1).uniform(n) * np.log(1e3))
        m /= m.sum()
    return x, y, z, m


CASES = [
    # kind, n, seed, r_cut, theta, n_leaf, n_crit
    ("uniform", 32768, 1, 3 / 32, 0.5, 10, 64),      # the plain-method box (32^3, mesh 32^3)
    ("nfw", 40000, 2, 0.06, 0.5, 10, 128),
    ("nfw", 20011, 3, 0.08, 0.8, 4, 37),             # ragged N, deep chains, odd n_crit
    ("uniform", 777, 4, 0.25, 0.3, 2, 5),            # tiny, n_leaf 2
    ("nfw", 30000, 5, 0.05, 1.0, 10, 300),
    ("nfw", 25000, 6, 0.06, 0.5, 300, 256),          # n_leaf above the flat build's window
]


def _ids(c):
    return f"{c[0]}-n{c[1]}-th{c[4]}-leaf{c[5]}-crit{c[6]}"


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_tree_and_lists_bit_identical(tp, orc, case):
    kind, n, seed, r_cut, theta, n_leaf, n_crit = case
    _say(f"tree/lists {_ids(case)}")
    x, y, z, m = _box(kind, n, seed)
    eps = r_cut / 60
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP64)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit)
    # keys and stable order
    gk, gi = tp.treepm_export_sorted(run.ctx)
    ok, oi = T.sorted()
    np.testing.assert_array_equal(gk, ok)
    np.testing.assert_array_equal(gi, oi)
    # nodes: same set of codes, same ranges, bitwise equal moments
    gn, on = tp.treepm_export_nodes(run.ctx), T.nodes()
    assert gn["code"].size == on["code"].size
    go, oo = np.argsort(gn["code"]), np.argsort(on["code"])
    for k in ("code", "first", "count", "nchild", "mass", "com"):
        np.testing.assert_array_equal(gn[k][go], on[k][oo], err_msg=k)
    # groups in key order
    gg, og = tp.treepm_export_groups(run.ctx), T.groups()
    for k in ("code", "first", "count", "lo", "hi", "xg"):
        np.testing.assert_array_equal(gg[k], og[k], err_msg=k)
    # lists: per group the same multiset of (kind, value)
    goff, gisc, gval = tp.treepm_export_lists(run.ctx)
    ooff, oisc, oval = T.lists()
    np.testing.assert_array_equal(np.diff(goff), np.diff(ooff))
    for g in range(og["code"].size):
        a = sorted(zip(gisc[goff[g]:goff[g + 1]].tolist(), gval[goff[g]:goff[g + 1]].tolist()))
        b = sorted(zip(oisc[ooff[g]:ooff[g + 1]].tolist(), oval[ooff[g]:ooff[g + 1]].tolist()))
        assert a == b, f"group {g}"
    assert run.stats.interactions == T.interactions()
    assert run.stats.n_cell_entries == int(oisc.sum())
    run.close()


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_fp64_force_matches_oracle(tp, orc, case):
    kind, n, seed, r_cut, theta, n_leaf, n_crit = case
    _say(f"fp64 force {_ids(case)}")
    x, y, z, m = _box(kind, n, seed)
    eps = r_cut / 60
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP64)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit)
    ref = np.stack(T.force())
    scale = T.error_scale()
    err = np.abs(run.acc - ref)
    assert np.all(err <= 1e-13 * scale[None, :] + 1e-300), float(np.max(err / (scale + 1e-300)))
    run.close()


@pytest.mark.parametrize("case", CASES[:3] + CASES[4:], ids=[_ids(c) for c in CASES[:3] + CASES[4:]])
def test_fp32_force_error_vs_fp64_oracle(tp, orc, case):
    kind, n, seed, r_cut, theta, n_leaf, n_crit = case
    _say(f"fp32 force {_ids(case)}")
    x, y, z, m = _box(kind, n, seed)
    eps = r_cut / 60
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP32,
              out64=True)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit)
    ref = np.stack(T.force())
    B = fp32_error_scale(T, x, y, z, m, eps)
    d = np.linalg.norm(run.acc - ref, axis=0)
    nr = np.linalg.norm(ref, axis=0)
    nz = nr > 0
    rel = d[nz] / nr[nz]
    rms = float(np.sqrt(np.mean(rel ** 2)))
    _say(f"  rms rel {rms:.3e} max rel {rel.max():.3e} p99 {np.quantile(rel, 0.99):.3e} "
         f"max |da|/(u B) {np.max(d / (2.0 ** -24 * B)):.3f}")
    assert rms <= 1e-6
    assert np.all(d[~nz] == 0.0)
    assert np.all(d <= 8 * 2.0 ** -24 * B)
    run.close()


def test_unequal_masses(tp, orc):
    """Masses over three decades on a clustered box with ragged N: node masses and centres of
    mass bit-identical, the same lists (the opening criterion measures from the centre of
    mass), the FP64 force to 1e-13 of the summed magnitudes and the FP32 force within its
    bound.  Every other parity case has equal masses."""
    _say("unequal masses")
    n, r_cut, theta, n_leaf, n_crit = 20011, 3 / 32, 0.5, 10, 64
    x, y, z, _ = boxgen.nfw_box(n, 50, 12)
    m = np.exp(boxgen.SplitMix64(13).uniform(n) * np.log(1e3))
    m /= m.sum()
    eps = r_cut / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit)
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP64)
    gn, on = tp.treepm_export_nodes(run.ctx), T.nodes()
    go, oo = np.argsort(gn["code"]), np.argsort(on["code"])
    for k in ("code", "count", "mass", "com"):
        np.testing.assert_array_equal(gn[k][go], on[k][oo], err_msg=k)
    goff, gisc, gval = tp.treepm_export_lists(run.ctx)
    ooff, oisc, oval = T.lists()
    np.testing.assert_array_equal(np.diff(goff), np.diff(ooff))
    for g in range(len(ooff) - 1):
        a = sorted(zip(gisc[goff[g]:goff[g + 1]].tolist(), gval[goff[g]:goff[g + 1]].tolist()))
        b = sorted(zip(oisc[ooff[g]:ooff[g + 1]].tolist(), oval[ooff[g]:ooff[g + 1]].tolist()))
        assert a == b, f"group {g}"
    ref = np.stack(T.force())
    scale = T.error_scale()
    err = np.abs(run.acc - ref)
    assert np.all(err <= 1e-13 * scale[None, :] + 1e-300), float(np.max(err / (scale + 1e-300)))
    run.close()
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP32,
              out64=True)
    B = fp32_error_scale(T, x, y, z, m, eps)
    d = np.linalg.norm(run.acc - ref, axis=0)
    _say(f"  fp32 max |da|/(u B) {np.max(d / (2.0 ** -24 * B)):.3f}")
    assert np.all(d <= 8 * 2.0 ** -24 * B)
    run.close()


def fp32_error_scale(T, x, y, z, m, eps):
    """B_i of the FP32 bound, from the oracle's groups and lists (FP64, numpy)."""
    k, idx = T.sorted()
    pos = np.stack([x, y, z], axis=1)[idx]
    nd = T.nodes()
    G = T.groups()
    off, isc, val = T.lists()
    code_to_node = {int(c): u for u, c in enumerate(nd["code"])}
    B = np.zeros(len(x))
    for g in range(G["code"].size):
        s, e = off[g], off[g + 1]
        cells = isc[s:e].astype(bool)
        src = np.empty((e - s, 3))
        sm = np.empty(e - s)
        pj = val[s:e][~cells].astype(np.int64)
        src[~cells] = np.stack([x[pj], y[pj], z[pj]], axis=1)
        sm[~cells] = m[pj]
        if cells.any():
            us = np.array([code_to_node[int(c)] for c in val[s:e][cells]])
            src[cells] = nd["com"][us]
            sm[cells] = nd["mass"][us]
        f0, c = int(G["first"][g]), int(G["count"][g])
        xi = pos[f0:f0 + c] - G["xg"][g]
        xj = src - G["xg"][g]
        xj -= np.floor(xj + 0.5)
        dd = xj[None, :, :] - xi[:, None, :]
        r2 = (dd * dd).sum(-1)
        w = np.abs(xi).max(1)[:, None] + np.abs(xj).max(1)[None, :] + np.sqrt(r2)
        B[idx[f0:f0 + c]] = (sm[None, :] * w / (r2 + eps * eps) ** 1.5).sum(1)
    return B


def test_theta_zero_equals_direct_sum(tp, orc):
    _say("theta=0 vs direct sum")
    x, y, z, m = boxgen.uniform_box(32768, 1)
    r_cut, eps = 3 / 32, 1 / 640
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, 0.0, 10, 64, tp.TREEPM_FP64)
    ref = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, eps))
    scale = np.max(np.linalg.norm(ref, axis=0))
    assert np.max(np.abs(run.acc - ref)) <= 1e-12 * scale
    run.close()


def test_deterministic_repeat(tp):
    _say("determinism")
    x, y, z, m = boxgen.nfw_box(50000, 80, 9)
    outs = []
    for prec in (tp.TREEPM_FP32, tp.TREEPM_FP64):
        a = Run(tp, x, y, z, m, 1.0, 0.06, 0.001, 0.5, 10, 96, prec)
        b = Run(tp, x, y, z, m, 1.0, 0.06, 0.001, 0.5, 10, 96, prec)
        np.testing.assert_array_equal(a.acc, b.acc)
        a.close(); b.close()


def test_host_buffers_and_fp32_output(tp, orc):
    _say("host buffers")
    x, y, z, m = boxgen.uniform_box(5000, 11)
    a = Run(tp, x, y, z, m, 1.0, 0.15, 0.002, 0.5, 10, 64, tp.TREEPM_FP32, out64=False, host=True)
    b = Run(tp, x, y, z, m, 1.0, 0.15, 0.002, 0.5, 10, 64, tp.TREEPM_FP32, out64=True)
    np.testing.assert_array_equal(a.acc, b.acc.astype(np.float32).astype(np.float64))
    a.close(); b.close()


def test_one_pass_walk_on_a_reused_context(tp, orc):
    """A context's later walks write the lists in one pass, into a pool sized from its previous
    walk; a box with more interactions than the previous one overflows that pool and is walked
    again in two passes.  Lists and FP64 forces must match the oracle on every path."""
    r_cut, theta, n_leaf, n_crit = 0.06, 0.5, 10, 128
    eps = r_cut / 60
    boxes = {"small": boxgen.nfw_box(8000, 20, 21), "big": boxgen.nfw_box(40000, 100, 2)}
    trees = {k: orc.Tree(*b, 1.0, r_cut, eps, theta, n_leaf, n_crit) for k, b in boxes.items()}
    p = tp.treepm_params(1.0, r_cut / 3.0, r_cut, eps, theta, n_leaf, n_crit, tp.TREEPM_FP64)
    ctx = tp.treepm_create(p, 0)
    tp.treepm_set_walk_passes(ctx, tp.TREEPM_WALK_ONE_PASS)  # at any box size
    try:
        for name in ("small", "small", "big", "big"):
            _say(f"reused context: {name} box")
            x, y, z, m = boxes[name]
            T = trees[name]
            tp.treepm_build(ctx, *[torch.from_numpy(a).cuda() for a in (x, y, z, m)])
            st = tp.treepm_walk(ctx)
            assert st.interactions == T.interactions()
            goff, gisc, gval = tp.treepm_export_lists(ctx)
            ooff, oisc, oval = T.lists()
            np.testing.assert_array_equal(np.diff(goff), np.diff(ooff))
            for g in range(ooff.size - 1):
                a = sorted(zip(gisc[goff[g]:goff[g + 1]].tolist(), gval[goff[g]:goff[g + 1]].tolist()))
                b = sorted(zip(oisc[ooff[g]:ooff[g + 1]].tolist(), oval[ooff[g]:ooff[g + 1]].tolist()))
                assert a == b, f"{name}: group {g}"
            acc = [torch.zeros(len(x), dtype=torch.float64, device="cuda") for _ in range(3)]
            tp.treepm_force_short(ctx, *acc)
            torch.cuda.synchronize()
            got = np.stack([t.cpu().numpy() for t in acc])
            ref = np.stack(T.force())
            assert np.all(np.abs(got - ref) <= 1e-13 * T.error_scale()[None, :] + 1e-300)
    finally:
        tp.treepm_destroy(ctx)


def test_walk_modes_give_the_same_lists(tp, orc):
    """Every walk mode (automatic: two passes for a box this small; one pass into the pool;
    always two passes) gives the oracle's lists and the same FP32 forces bit for bit, on the
    first and on later walks of a context; other modes are rejected."""
    x, y, z, m = boxgen.nfw_box(30000, 60, 41)
    r_cut, eps = 0.07, 0.07 / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.5, 10, 64)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    p = tp.treepm_params(1.0, r_cut / 3.0, r_cut, eps, 0.5, 10, 64, tp.TREEPM_FP32)
    ref = None
    for mode in (tp.TREEPM_WALK_AUTO, tp.TREEPM_WALK_ONE_PASS, tp.TREEPM_WALK_TWO_PASS):
        ctx = tp.treepm_create(p, 0)
        try:
            tp.treepm_set_walk_passes(ctx, mode)
            for rep in range(3):
                _say(f"walk mode {mode} walk {rep}")
                tp.treepm_build(ctx, *dev)
                st = tp.treepm_walk(ctx)
                assert st.interactions == T.interactions()
                _assert_lists_equal(tp, ctx, T, f"mode {mode} walk {rep}")
                acc = [torch.zeros(30000, dtype=torch.float32, device="cuda") for _ in range(3)]
                tp.treepm_force_short(ctx, *acc)
                torch.cuda.synchronize()
                got = np.stack([t.cpu().numpy() for t in acc])
                if ref is None:
                    ref = got
                np.testing.assert_array_equal(got, ref)
            for bad in (-1, 3):
                with pytest.raises(tp.TreePMError) as e:
                    tp.treepm_set_walk_passes(ctx, bad)
                assert e.value.code == -1
        finally:
            tp.treepm_destroy(ctx)


def _assert_lists_equal(tp, ctx, T, what):
    goff, gisc, gval = tp.treepm_export_lists(ctx)
    ooff, oisc, oval = T.lists()
    np.testing.assert_array_equal(np.diff(goff), np.diff(ooff))
    for g in range(ooff.size - 1):
        a = sorted(zip(gisc[goff[g]:goff[g + 1]].tolist(), gval[goff[g]:goff[g + 1]].tolist()))
        b = sorted(zip(oisc[ooff[g]:ooff[g + 1]].tolist(), oval[ooff[g]:ooff[g + 1]].tolist()))
        assert a == b, f"{what}: group {g}"
    return int(oisc.sum())


OPEN_CASES = [
    # kind, n, seed, r_cut, theta_0, theta_max, n_leaf, n_crit
    ("uniform", 32768, 1, 3 / 32, 0.05, 0.6, 10, 64),  # the uniform-limit pin's setting
    ("nfw", 40000, 2, 0.06, 0.25, 0.8, 10, 128),
    ("nfw", 20011, 3, 0.08, 0.15, 1.0, 4, 37),        # ragged N, odd n_crit, cap 1
    ("nfw", 30000, 5, 0.05, 0.3, 0.0, 10, 300),       # cap 0: no cell is ever accepted
]


@pytest.mark.parametrize("case", OPEN_CASES,
                         ids=[f"{c[0]}-n{c[1]}-th0{c[4]}-max{c[5]}" for c in OPEN_CASES])
def test_distance_opening_parity(tp, orc, case):
    """The distance-dependent angle of eq. (12): lists bit-identical to the oracle's on the
    two-pass walk of a fresh context and on the one-pass walk of the same context; FP64 and
    FP32 forces to the bars of the fixed-angle tests."""
    kind, n, seed, r_cut, th0, tmax, n_leaf, n_crit = case
    x, y, z, m = _box(kind, n, seed)
    eps = r_cut / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, th0, n_leaf, n_crit, opening=1, theta_max=tmax)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    for prec in (tp.TREEPM_FP64, tp.TREEPM_FP32):
        p = tp.make_params(1.0, r_cut / 3.0, r_cut, eps, th0, n_leaf, n_crit, prec,
                           opening=tp.TREEPM_OPEN_DISTANCE, theta_max=tmax)
        ctx = tp.treepm_create(p, 0)
        tp.treepm_set_walk_passes(ctx, tp.TREEPM_WALK_ONE_PASS)  # the second walk: one pass
        try:
            for walk in ("two-pass", "one-pass"):
                _say(f"theta(r) {kind} n={n} th0={th0} max={tmax} prec={prec} {walk}")
                tp.treepm_build(ctx, *dev)
                st = tp.treepm_walk(ctx)
                assert st.interactions == T.interactions()
                ncell = _assert_lists_equal(tp, ctx, T, walk)
                assert st.n_cell_entries == ncell
                if tmax == 0.0:
                    assert ncell == 0
                acc = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
                tp.treepm_force_short(ctx, *acc)
                torch.cuda.synchronize()
                got = np.stack([t.cpu().numpy() for t in acc])
                ref = np.stack(T.force())
                if prec == tp.TREEPM_FP64:
                    assert np.all(np.abs(got - ref) <= 1e-13 * T.error_scale()[None, :] + 1e-300)
                else:
                    d = np.linalg.norm(got - ref, axis=0)
                    nr = np.linalg.norm(ref, axis=0)
                    nz = nr > 0
                    rms = float(np.sqrt(np.mean((d[nz] / nr[nz]) ** 2)))
                    _say(f"  fp32 rms rel {rms:.3e}")
                    assert rms <= 1e-6
                    assert np.all(d[~nz] == 0.0)
                    if walk == "two-pass":
                        B = fp32_error_scale(T, x, y, z, m, eps)
                        assert np.all(d <= 8 * 2.0 ** -24 * B)
        finally:
            tp.treepm_destroy(ctx)


def _clumped_box(n_uniform, clumps, seed):
    """Uniform particles plus clumps, each inside one cell of side 2^-11, so each clump's keys
    share their high bits and differ in the low ones; clump sizes are given.  Every fifth
    clump member repeats its predecessor's position exactly (equal keys, ordered by index)."""
    rng = boxgen.SplitMix64(seed)
    parts = [rng.uniform(3 * n_uniform).reshape(3, n_uniform)]
    for size in clumps:
        corner = np.floor(rng.uniform(3) * 2048.0) / 2048.0
        off = rng.uniform(3 * size).reshape(3, size) * (1.0 / 2048.0)
        off[:, 4::5] = off[:, 3::5][:, : off[:, 4::5].shape[1]]
        parts.append(corner[:, None] + off)
    p = np.concatenate(parts, axis=1)
    perm = np.argsort(rng.next_u64(p.shape[1]), kind="stable")
    x, y, z = (np.ascontiguousarray(p[a, perm]) for a in range(3))
    return x, y, z, np.full(x.size, 1.0 / x.size)


@pytest.mark.parametrize("clumps", [[2, 3, 17, 40, 64, 64, 5] * 6, [2, 64, 65, 300]],
                         ids=["runs-up-to-64", "runs-over-64"])
def test_sort_order_with_clumps(tp, orc, clumps):
    """Keys sorted by their high bits, then runs of equal high bits in place (longer runs fall
    back to sorting all bits): the order must still be (key, input index) exactly."""
    _say(f"sort order, clumps {sorted(set(clumps))}")
    x, y, z, m = _clumped_box(3000, clumps, 91)
    run = Run(tp, x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64, tp.TREEPM_FP64)
    T = orc.Tree(x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64)
    gk, gi = tp.treepm_export_sorted(run.ctx)
    ok, oi = T.sorted()
    np.testing.assert_array_equal(gk, ok)
    np.testing.assert_array_equal(gi, oi)
    gn, on = tp.treepm_export_nodes(run.ctx), T.nodes()
    go, oo = np.argsort(gn["code"]), np.argsort(on["code"])
    for k in ("code", "first", "count", "mass", "com"):
        np.testing.assert_array_equal(gn[k][go], on[k][oo], err_msg=k)
    run.close()


def test_edge_cases(tp, orc):
    _say("edge cases")
    # a single particle feels nothing
    r = Run(tp, np.array([0.3]), np.array([0.4]), np.array([0.5]), np.array([1.0]), 1.0, 0.3,
            0.01, 0.5, 10, 64, tp.TREEPM_FP64)
    assert np.all(r.acc == 0.0)
    r.close()
    # fewer particles than n_leaf and n_crit: the root is the only node and group
    x, y, z, m = boxgen.uniform_box(7, 3)
    r = Run(tp, x, y, z, m, 1.0, 0.3, 0.01, 0.5, 10, 64, tp.TREEPM_FP64)
    assert r.stats.n_nodes == 1 and r.stats.n_groups == 1
    ref = np.stack(orc.direct_brute(x, y, z, m, 1.0, 0.3, 0.01))
    np.testing.assert_allclose(r.acc, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    r.close()
    # many coincident particles: level-21 leaves holding more than n_leaf
    n = 3000
    x, y, z, m = boxgen.uniform_box(n, 5)
    x[:500] = 0.25; y[:500] = 0.5; z[:500] = 0.75
    r = Run(tp, x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64, tp.TREEPM_FP64)
    T = orc.Tree(x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64)
    assert r.stats.max_level == 21
    gn, on = tp.treepm_export_nodes(r.ctx), T.nodes()
    go, oo = np.argsort(gn["code"]), np.argsort(on["code"])
    for k in ("code", "first", "count", "nchild", "mass", "com"):
        np.testing.assert_array_equal(gn[k][go], on[k][oo], err_msg=k)
    assert on["count"].max() == n  # the root; the clump's level-21 leaf holds 500
    ref = np.stack(T.force())
    assert np.all(np.abs(r.acc - ref) <= 1e-13 * T.error_scale()[None, :] + 1e-300)
    r.close()


def test_error_paths(tp):
    _say("error paths")
    p = tp.treepm_params(1.0, 0.1, 0.3, 0.01, 0.5, 10, 64, tp.TREEPM_FP64)
    ctx = tp.treepm_create(p, 0)
    x, y, z, m = (torch.from_numpy(a).cuda() for a in boxgen.uniform_box(100, 1))
    a = [torch.zeros(100, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_walk(ctx)
    assert e.value.code == -5
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_force_short(ctx, *a)
    assert e.value.code == -5
    xb = x.clone(); xb[7] = 1.0
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_build(ctx, xb, y, z, m)
    assert e.value.code == -2
    xb = x.clone(); xb[3] = -1e-9
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_build(ctx, xb, y, z, m)
    assert e.value.code == -2
    mb = m.clone(); mb[5] = float("nan")
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_build(ctx, x, y, z, mb)
    assert e.value.code == -1
    mb = m.clone(); mb[5] = 0.0
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_build(ctx, x, y, z, mb)
    assert e.value.code == -1
    # a failed build leaves the context empty
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_walk(ctx)
    assert e.value.code == -5
    # and a good build afterwards works
    tp.treepm_build(ctx, x, y, z, m)
    tp.treepm_walk(ctx)
    tp.treepm_force_short(ctx, *a)
    tp.treepm_destroy(ctx)
    # FP32 path refuses a group too large for one image per entry (root group, r_cut = 0.3)
    p32 = tp.treepm_params(1.0, 0.1, 0.3, 0.01, 0.5, 10, 64, tp.TREEPM_FP32)
    ctx = tp.treepm_create(p32, 0)
    tp.treepm_build(ctx, x, y, z, m)
    tp.treepm_walk(ctx)
    with pytest.raises(tp.TreePMError) as e:
        tp.treepm_force_short(ctx, *a)
    assert e.value.code == -1
    tp.treepm_destroy(ctx)
    # opening criterion: unknown mode, cap outside [0, 1]
    for bad in (dict(opening=2), dict(opening=1, theta_max=1.5),
                dict(opening=1, theta_max=float("nan")), dict(opening=1, theta_max=-0.1)):
        q = tp.make_params(1.0, 0.1, 0.3, 0.01, 0.5, 10, 64, tp.TREEPM_FP64, **bad)
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_create(q, 0)
        assert e.value.code == -1, bad


def test_autotune_picks_a_candidate_and_leaves_a_walked_box(tp, orc):
    _say("autotune")
    x, y, z, m = boxgen.nfw_box(60000, 100, 13)
    r_cut, eps = 0.05, 0.05 / 60
    p = tp.treepm_params(1.0, r_cut / 3, r_cut, eps, 0.5, 10, 64, tp.TREEPM_FP32)
    ctx = tp.treepm_create(p, 0)
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    best, ms = tp.treepm_autotune(ctx, *dev, [32, 96, 200])
    assert best in (32, 96, 200) and ms > 0
    a = [torch.zeros(len(x), dtype=torch.float64, device="cuda") for _ in range(3)]
    tp.treepm_force_short(ctx, *a)      # the box is built and walked with the winner
    got = np.stack([t.cpu().numpy() for t in a])
    tp.treepm_destroy(ctx)
    ref = Run(tp, x, y, z, m, 1.0, r_cut, eps, 0.5, 10, best, tp.TREEPM_FP32)
    np.testing.assert_array_equal(got, ref.acc)
    ref.close()


QUAD_CASES = [
    ("uniform", 32768, 1, 3 / 32, 0.5, 10, 64),
    ("nfw", 40000, 2, 0.06, 0.5, 10, 128),
    ("nfw", 20011, 3, 0.08, 0.8, 4, 37),
    ("nfw-masses", 20011, 14, 3 / 32, 0.6, 10, 64),  # second moments weighted by mass
]


@pytest.mark.parametrize("case", QUAD_CASES, ids=[_ids(c) for c in QUAD_CASES])
def test_quadrupole_parity(tp, orc, case):
    """Cells with their second-order terms (Section 4.1): FP64 forces to the fixed-angle bar,
    1e-13 of the summed magnitudes (the oracle evaluates the expanded eq. (2) and its
    derivatives, the kernel the factored second branch; measured up to 6e-15), FP32 forces to
    the FP32 bar; the lists are the fixed-angle ones."""
    kind, n, seed, r_cut, theta, n_leaf, n_crit = case
    x, y, z, m = _box(kind, n, seed)
    eps = r_cut / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit, quadrupole=True)
    ref = np.stack(T.force())
    scale = T.error_scale()
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    for prec in (tp.TREEPM_FP64, tp.TREEPM_FP32):
        _say(f"quadrupole {_ids(case)} prec={prec}")
        p = tp.make_params(1.0, r_cut / 3.0, r_cut, eps, theta, n_leaf, n_crit, prec,
                           quadrupole=1)
        ctx = tp.treepm_create(p, 0)
        try:
            tp.treepm_build(ctx, *dev)
            st = tp.treepm_walk(ctx)
            assert st.interactions == T.interactions()
            acc = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
            tp.treepm_force_short(ctx, *acc)
            torch.cuda.synchronize()
            got = np.stack([t.cpu().numpy() for t in acc])
        finally:
            tp.treepm_destroy(ctx)
        if prec == tp.TREEPM_FP64:
            r = np.max(np.abs(got - ref) / (scale[None, :] + 1e-300))
            _say(f"  fp64 max |da| / scale {r:.2e}")
            assert r <= 1e-13
        else:
            d = np.linalg.norm(got - ref, axis=0)
            nr = np.linalg.norm(ref, axis=0)
            nz = nr > 0
            rms = float(np.sqrt(np.mean((d[nz] / nr[nz]) ** 2)))
            _say(f"  fp32 rms rel {rms:.3e}")
            assert rms <= 1e-6
            assert np.all(d[~nz] == 0.0)


def test_quadrupole_with_distance_opening(tp, orc):
    """Both Section 4.1 options at once: lists under theta(d) (theta_0 = 0.25, cap 0.8) with the
    cells' second-order terms; FP64 and FP32 bars as above."""
    x, y, z, m = _box("nfw", 40000, 2)
    r_cut, th0, tmax = 0.06, 0.25, 0.8
    eps = r_cut / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, th0, 10, 128, opening=1, theta_max=tmax,
                 quadrupole=True)
    ref = np.stack(T.force())
    scale = T.error_scale()
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    for prec in (tp.TREEPM_FP64, tp.TREEPM_FP32):
        _say(f"quadrupole + theta(r) prec={prec}")
        p = tp.make_params(1.0, r_cut / 3.0, r_cut, eps, th0, 10, 128, prec,
                           opening=tp.TREEPM_OPEN_DISTANCE, theta_max=tmax, quadrupole=1)
        ctx = tp.treepm_create(p, 0)
        try:
            tp.treepm_build(ctx, *dev)
            st = tp.treepm_walk(ctx)
            assert st.interactions == T.interactions()
            _assert_lists_equal(tp, ctx, T, "theta(r) + quadrupole")
            acc = [torch.zeros(len(x), dtype=torch.float64, device="cuda") for _ in range(3)]
            tp.treepm_force_short(ctx, *acc)
            torch.cuda.synchronize()
            got = np.stack([t.cpu().numpy() for t in acc])
        finally:
            tp.treepm_destroy(ctx)
        if prec == tp.TREEPM_FP64:
            assert np.all(np.abs(got - ref) <= 1e-13 * scale[None, :] + 1e-300)
        else:
            d = np.linalg.norm(got - ref, axis=0)
            nr = np.linalg.norm(ref, axis=0)
            nz = nr > 0
            assert float(np.sqrt(np.mean((d[nz] / nr[nz]) ** 2))) <= 1e-6


@pytest.mark.parametrize("n", [1, 2, 9])
def test_quadrupole_tiny_boxes(tp, orc, n):
    """Quadrupole cells on boxes of a few particles (few or no cell entries), FP64 output."""
    x, y, z, m = boxgen.uniform_box(n, 60 + n)
    r_cut = 0.3
    T = orc.Tree(x, y, z, m, 1.0, r_cut, 0.002, 0.8, 2, 2, quadrupole=True)
    ref = np.stack(T.force())
    p = tp.make_params(1.0, r_cut / 3, r_cut, 0.002, 0.8, 2, 2, tp.TREEPM_FP64, quadrupole=1)
    ctx = tp.treepm_create(p, 0)
    try:
        tp.treepm_build(ctx, *[torch.from_numpy(a).cuda() for a in (x, y, z, m)])
        tp.treepm_walk(ctx)
        acc = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        tp.treepm_force_short(ctx, *acc)
        torch.cuda.synchronize()
        got = np.stack([t.cpu().numpy() for t in acc])
    finally:
        tp.treepm_destroy(ctx)
    assert np.all(np.abs(got - ref) <= 1e-13 * T.error_scale()[None, :] + 1e-300)


def test_sort_fallback_run_over_2048(tp, orc):
    """More than 2048 particles share one level-13 cell (the same key bits 24-62), which is
    longer than the in-place sort of runs handles, so the build sorts all key bits instead:
    the order, the nodes and the FP64 force must still equal the oracle's."""
    rng = boxgen.SplitMix64(4242)
    n_bg, n_cl = 3000, 2600
    bg = rng.uniform(3 * n_bg).reshape(3, n_bg)
    corner = np.array([1234.0, 4321.0, 777.0]) / 8192.0
    cl = corner[:, None] + rng.uniform(3 * n_cl).reshape(3, n_cl) * (1.0 / 8192.0)
    cl[:, 5::7] = cl[:, 4::7][:, : cl[:, 5::7].shape[1]]  # some exactly equal keys too
    p = np.concatenate([bg, cl], axis=1)
    perm = np.argsort(rng.next_u64(p.shape[1]), kind="stable")
    x, y, z = (np.ascontiguousarray(p[a, perm]) for a in range(3))
    m = np.full(x.size, 1.0 / x.size)
    T = orc.Tree(x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64)
    ok, oi = T.sorted()
    hi = ok >> np.uint64(24)
    runs = np.diff(np.flatnonzero(np.concatenate([[True], hi[1:] != hi[:-1], [True]])))
    _say(f"sort fallback: longest run of equal high key bits {runs.max()}")
    assert runs.max() > 2048  # the case the in-place run sort does not take
    run = Run(tp, x, y, z, m, 1.0, 0.1, 0.002, 0.5, 10, 64, tp.TREEPM_FP64)
    gk, gi = tp.treepm_export_sorted(run.ctx)
    np.testing.assert_array_equal(gk, ok)
    np.testing.assert_array_equal(gi, oi)
    gn, on = tp.treepm_export_nodes(run.ctx), T.nodes()
    go, oo = np.argsort(gn["code"]), np.argsort(on["code"])
    for k in ("code", "first", "count", "nchild", "mass", "com"):
        np.testing.assert_array_equal(gn[k][go], on[k][oo], err_msg=k)
    assert run.stats.interactions == T.interactions()
    ref = np.stack(T.force())
    assert np.all(np.abs(run.acc - ref) <= 1e-13 * T.error_scale()[None, :] + 1e-300)
    run.close()


def _check_fp32(run, T, x, y, z, m, eps):
    ref = np.stack(T.force())
    B = fp32_error_scale(T, x, y, z, m, eps)
    d = np.linalg.norm(run.acc - ref, axis=0)
    nr = np.linalg.norm(ref, axis=0)
    nz = nr > 0
    rel = d[nz] / nr[nz]
    rms = float(np.sqrt(np.mean(rel ** 2)))
    _say(f"  rms rel {rms:.3e} max rel {rel.max():.3e} "
         f"max |da|/(u B) {np.max(d / (2.0 ** -24 * B)):.3f}")
    assert rms <= 1e-6
    assert np.all(d[~nz] == 0.0)
    assert np.all(d <= 8 * 2.0 ** -24 * B)


def test_fp32_groups_over_512(tp, orc):
    """n_crit = 600: groups of 513-600 particles take the FP32 kernel's widest layout (one
    stream, eight particles per lane) in chunks of 512 particles; lists and forces as for
    every other group."""
    n, seed, r_cut, n_crit = 60000, 7, 0.06, 600
    x, y, z, m = boxgen.nfw_box(n, n // 400, seed)
    eps = r_cut / 60
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.5, 10, n_crit)
    big = int((T.groups()["count"] > 512).sum())
    _say(f"fp32 groups over 512: {big} of {T.n_groups} groups")
    assert big > 10
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, 0.5, 10, n_crit, tp.TREEPM_FP32)
    assert run.stats.interactions == T.interactions()
    assert run.stats.max_group == int(T.groups()["count"].max())
    _check_fp32(run, T, x, y, z, m, eps)
    run.close()


def test_fp32_coincident_clump_of_700(tp, orc):
    """700 particles at one position make a level-21 leaf of 700 (a group above n_crit and
    above 512): the FP32 kernel runs it in two chunks; pairs at zero separation add
    nothing."""
    n = 6000
    x, y, z, m = boxgen.uniform_box(n, 17)
    x[100:800] = 0.3125; y[100:800] = 0.6; z[100:800] = 0.9
    r_cut, eps = 0.1, 0.002
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.5, 10, 64)
    assert int(T.groups()["count"].max()) == 700
    _say("fp32 coincident clump of 700")
    run = Run(tp, x, y, z, m, 1.0, r_cut, eps, 0.5, 10, 64, tp.TREEPM_FP32)
    assert run.stats.max_group == 700 and run.stats.max_level == 21
    assert run.stats.interactions == T.interactions()
    _check_fp32(run, T, x, y, z, m, eps)
    run.close()
