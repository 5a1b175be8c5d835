"""Pins of the oracle's reference tree, groups and interaction lists (no GPU).

Section 2.2 steps 2 and 5 (local tree, Barnes' interaction-list walk), Section 3.1.2 (N_leaf
stopping rule, N_crit grouping), Section 2.2 step 3 (opening criterion and cutoff both
measured from the surface of the receiving region).  The method is an approximation, so the
pins are: hand-computed keys, structural invariants, a brute-force frontier built from all
nodes without recursion, geometric checks of every pruned and accepted node against the
particles themselves, exact coverage of every particle within r_cut, and the theta -> 0
limit equal to the exact direct sum.  The distance-dependent opening angle of Section 4.1
(eq. 12) is pinned by closed-form values of the angle, its cap, the same brute-force
frontier, and the paper's uniform-density claim (less error at no more cost).
"""
import math

import numpy as np
import pytest

import boxgen


def decode(code: int):
    """Node code (1 << 3l) | prefix -> (level, ix, iy, iz)."""
    lev = (int(code).bit_length() - 1) // 3
    pre = int(code) ^ (1 << (3 * lev))
    ix = iy = iz = 0
    for b in range(lev):
        d = (pre >> (3 * (lev - 1 - b))) & 7
        ix = 2 * ix + ((d >> 2) & 1)
        iy = 2 * iy + ((d >> 1) & 1)
        iz = 2 * iz + (d & 1)
    return lev, ix, iy, iz


def test_keys_hand_computed(orc):
    # x is the most significant bit of each triplet, then y, then z.
    assert orc.key(0.5, 0.0, 0.0) == 1 << 62
    assert orc.key(0.0, 0.5, 0.0) == 1 << 61
    assert orc.key(0.0, 0.0, 0.5) == 1 << 60
    assert orc.key(0.0, 0.0, 0.0) == 0
    top = 1.0 - 2.0 ** -21
    assert orc.key(top, top, top) == (1 << 63) - 1
    # the lowest triplet: one cell of 2^-21 along each axis
    assert orc.key(2.0 ** -21, 0.0, 0.0) == 4
    assert orc.key(0.0, 2.0 ** -21, 2.0 ** -21) == 3
    # the quantisation clamps at 2^21 - 1 (x just below L rounds to the top cell)
    assert orc.key(np.nextafter(1.0, 0.0), 0.0, 0.0) == orc.key(top, 0.0, 0.0)
    # another box size: key depends on x / L only
    assert orc.key(1.5, 0.75, 0.0, 3.0) == orc.key(0.5, 0.25, 0.0, 1.0)


def test_keys_decode_to_cells(orc):
    x, y, z, _ = boxgen.uniform_box(200, 3)
    for i in range(200):
        k = orc.key(x[i], y[i], z[i])
        lev, ix, iy, iz = decode((1 << 63) | k)
        assert lev == 21
        assert (ix, iy, iz) == tuple(int(math.floor(p * 2 ** 21)) for p in (x[i], y[i], z[i]))


def _tree(orc, n, seed, theta=0.5, n_leaf=4, n_crit=24, r_cut=0.2, eps=0.003, kind="nfw"):
    if kind == "nfw":
        x, y, z, m = boxgen.nfw_box(n, max(1, n // 100), seed)
    else:
        x, y, z, m = boxgen.uniform_box(n, seed)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, n_leaf, n_crit)
    return T, (x, y, z, m)


def test_sort_is_stable_key_sort(orc):
    # coarse positions force many equal keys; ties must keep input order
    rng = boxgen.SplitMix64(9)
    n = 3000
    x = np.floor(rng.uniform(n) * 4) / 4
    y = np.floor(rng.uniform(n) * 4) / 4
    z = np.floor(rng.uniform(n) * 4) / 4
    T = orc.Tree(x, y, z, np.full(n, 1.0 / n), 1.0, 0.2, 0.01, 0.5, 10, 64)
    k, idx = T.sorted()
    keys = np.array([orc.key(a, b, c) for a, b, c in zip(x, y, z)], dtype=np.uint64)
    ref = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(idx, ref)
    np.testing.assert_array_equal(k, keys[ref])


@pytest.mark.parametrize("seed,n_leaf", [(1, 2), (2, 4), (3, 10)])
def test_tree_invariants(orc, seed, n_leaf):
    T, (x, y, z, m) = _tree(orc, 1500, seed, n_leaf=n_leaf)
    k, idx = T.sorted()
    nd = T.nodes()
    n_nodes = nd["code"].size
    leaf_cover = np.zeros(T.n, dtype=np.int64)
    for u in range(n_nodes):
        lev, ix, iy, iz = decode(nd["code"][u])
        f, c = int(nd["first"][u]), int(nd["count"][u])
        assert c >= 1
        # every particle of the node shares its key prefix, and the neighbours outside do not
        pre = int(nd["code"][u]) ^ (1 << (3 * lev))
        sh = 3 * (21 - lev)
        assert all((int(kk) >> sh) == pre for kk in k[f:f + c])
        if f > 0:
            assert (int(k[f - 1]) >> sh) != pre
        if f + c < T.n:
            assert (int(k[f + c]) >> sh) != pre
        # mass is the sum of the particle masses; com lies inside the cube
        msum = float(np.sum(m[idx[f:f + c]]))
        assert nd["mass"][u] == pytest.approx(msum, rel=1e-13)
        l = 2.0 ** -lev
        lo = np.array([ix, iy, iz]) * l
        assert np.all(nd["com"][u] >= lo - 1e-15) and np.all(nd["com"][u] <= lo + l + 1e-15)
        # subdivision rule: leaf iff count < n_leaf or level 21
        is_leaf = nd["nchild"][u] == 0
        assert is_leaf == (c < n_leaf or lev == 21)
        if is_leaf:
            leaf_cover[f:f + c] += 1
    assert np.all(leaf_cover == 1)  # leaves partition the particles
    # children: codes at level+1 whose parent code is u, counts summing to the parent
    codes = {int(c): u for u, c in enumerate(nd["code"])}
    for u in range(n_nodes):
        if nd["nchild"][u] == 0:
            continue
        kids = [codes[(int(nd["code"][u]) << 3) | o] for o in range(8)
                if ((int(nd["code"][u]) << 3) | o) in codes]
        assert len(kids) == nd["nchild"][u]
        assert sum(int(nd["count"][v]) for v in kids) == nd["count"][u]


def test_groups_rule(orc):
    n_crit = 24
    T, (x, y, z, m) = _tree(orc, 3000, 4, n_crit=n_crit)
    nd = T.nodes()
    codes = {int(c): u for u, c in enumerate(nd["code"])}
    G = T.groups()
    cover = np.zeros(T.n, dtype=np.int64)
    k, idx = T.sorted()
    pos = np.stack([x, y, z], axis=1)[idx]
    for g in range(G["code"].size):
        u = codes[int(G["code"][g])]
        f, c = int(G["first"][g]), int(G["count"][g])
        assert c == nd["count"][u] and f == nd["first"][u]
        assert c <= n_crit or nd["nchild"][u] == 0
        if nd["code"][u] != 1:
            parent = codes[int(nd["code"][u]) >> 3]
            assert nd["count"][parent] > n_crit
        cover[f:f + c] += 1
        np.testing.assert_array_equal(G["lo"][g], pos[f:f + c].min(axis=0))
        np.testing.assert_array_equal(G["hi"][g], pos[f:f + c].max(axis=0))
        lev, ix, iy, iz = decode(G["code"][g])
        np.testing.assert_array_equal(G["xg"][g], (np.array([ix, iy, iz]) + 0.5) * 2.0 ** -lev)
    assert np.all(cover == 1)
    assert np.all(np.diff(G["first"]) > 0)  # key order


def _min_image(d):
    return d - np.floor(d + 0.5)


def _frontier_check(orc, T, pos_in, m_in, theta, r_cut, theta_of_d=None):
    """Rebuild each group's list from all nodes without recursion and check every entry
    geometrically against the particles.  theta_of_d: the angle as a function of the node's
    distance d from the group's bbox (distance-dependent opening); None = theta fixed."""
    k, idx = T.sorted()
    pos = pos_in[idx]
    nd = T.nodes()
    G = T.groups()
    off, isc, val = T.lists()
    n_nodes = nd["code"].size
    lev = np.array([decode(c)[0] for c in nd["code"]])
    cube = np.array([decode(c)[1:] for c in nd["code"]], dtype=np.float64)
    side = 2.0 ** -lev
    centre = (cube + 0.5) * side[:, None]
    codes = {int(c): u for u, c in enumerate(nd["code"])}
    ancestors = []
    for u in range(n_nodes):
        a, c = [], int(nd["code"][u])
        while c != 1:
            c >>= 3
            a.append(codes[c])
        ancestors.append(a)
    th2, rc2 = theta * theta, r_cut * r_cut
    total_inter = 0
    for g in range(G["code"].size):
        lo, hi = G["lo"][g], G["hi"][g]
        cg, hg = (lo + hi) * 0.5, (hi - lo) * 0.5
        gap = np.maximum(0.0, np.abs(_min_image(centre - cg)) - (side[:, None] * 0.5 + hg))
        Gs = (gap * gap).sum(axis=1)
        P = Gs >= rc2
        dc = np.maximum(0.0, np.abs(_min_image(nd["com"] - cg)) - hg)
        Ds = (dc * dc).sum(axis=1)
        if theta_of_d is None:
            thn = np.full(n_nodes, theta)
            th2n = np.full(n_nodes, th2)
        else:
            thn = np.array([theta_of_d(math.sqrt(v)) for v in Ds])
            th2n = thn * thn
        A = (side * side < th2n * Ds) & (Gs > 0.0) & ~P
        opened = ~A & ~P
        live = np.array([all(opened[a] for a in ancestors[u]) for u in range(n_nodes)])
        exp_cells = {int(nd["code"][u]) for u in np.nonzero(live & A)[0]}
        exp_parts = set()
        for u in np.nonzero(live & opened & (nd["nchild"] == 0))[0]:
            exp_parts.update(int(i) for i in idx[nd["first"][u]:nd["first"][u] + nd["count"][u]])
        s, e = off[g], off[g + 1]
        got_cells = [int(v) for v, c in zip(val[s:e], isc[s:e]) if c]
        got_parts = [int(v) for v, c in zip(val[s:e], isc[s:e]) if not c]
        assert len(set(got_cells)) == len(got_cells) and set(got_cells) == exp_cells
        assert len(set(got_parts)) == len(got_parts) and set(got_parts) == exp_parts
        total_inter += int(G["count"][g]) * (e - s)
        # geometry against the particles themselves
        gpos = pos[G["first"][g]:G["first"][g] + G["count"][g]]
        covered = np.zeros(T.n, dtype=np.int64)  # in sorted order
        for u in np.nonzero(live & A)[0]:
            f, c = int(nd["first"][u]), int(nd["count"][u])
            covered[f:f + c] += 1
            # accepted: side/theta < distance from com to the nearest group particle
            dmin = np.sqrt((_min_image(gpos - nd["com"][u]) ** 2).sum(axis=1)).min()
            assert side[u] < thn[u] * dmin
        for u in np.nonzero(live & P)[0]:
            f, c = int(nd["first"][u]), int(nd["count"][u])
            # pruned: every particle of the node is at least r_cut from every group particle
            d = _min_image(pos[f:f + c][:, None, :] - gpos[None, :, :])
            assert np.sqrt((d * d).sum(axis=2)).min() >= r_cut
        inv = np.empty(T.n, dtype=np.int64)
        inv[idx] = np.arange(T.n)
        covered[inv[np.array(sorted(exp_parts), dtype=np.int64)]] += 1
        # every particle within r_cut of the group is covered exactly once, none twice
        d = _min_image(pos[:, None, :] - gpos[None, :, :])
        near = np.sqrt((d * d).sum(axis=2)).min(axis=1) < r_cut
        assert np.all(covered[near] == 1)
        assert np.all(covered <= 1)
        # mass partition: list mass + pruned frontier mass = total mass
        mlist = sum(nd["mass"][codes[c]] for c in got_cells) + m_in[got_parts].sum()
        mpruned = nd["mass"][live & P].sum()
        assert mlist + mpruned == pytest.approx(m_in.sum(), rel=1e-12)
    assert total_inter == T.interactions()


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 0.8, 1.0])
def test_lists_equal_brute_force_frontier(orc, theta):
    n, r_cut = 400, 0.2
    T, (x, y, z, m) = _tree(orc, n, 5, theta=theta, n_leaf=3, n_crit=20, r_cut=r_cut)
    _frontier_check(orc, T, np.stack([x, y, z], axis=1), m, theta, r_cut)


def test_lists_uniform_box(orc):
    T, (x, y, z, m) = _tree(orc, 512, 6, theta=0.6, n_leaf=4, n_crit=16, r_cut=0.3,
                            kind="uniform")
    _frontier_check(orc, T, np.stack([x, y, z], axis=1), m, 0.6, 0.3)


@pytest.mark.parametrize("kind,seed", [("uniform", 7), ("nfw", 8)])
def test_theta_zero_is_direct_sum(orc, kind, seed):
    n, r_cut, eps = 6000, 0.1, 0.002
    T, (x, y, z, m) = _tree(orc, n, seed, theta=0.0, n_leaf=10, n_crit=64, r_cut=r_cut,
                            eps=eps, kind=kind)
    a = np.stack(T.force())
    b = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, eps))
    # condition-aware: compare against the scale of the largest accelerations
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.linalg.norm(b, axis=0))
    off, isc, val = T.lists()
    assert not isc.any()


def test_small_theta_without_cells_is_direct_sum(orc):
    """theta <= l_min/(r_cut + sqrt(3) l_min) can never accept a node, so the list force is
    the direct sum."""
    n, r_cut, eps = 3000, 0.1, 0.002
    x, y, z, m = boxgen.uniform_box(n, 9)
    T0 = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.0, 10, 64)
    lev = max(decode(c)[0] for c in T0.nodes()["code"])
    lmin = 2.0 ** -lev
    theta = lmin / (r_cut + math.sqrt(3.0) * lmin)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, theta, 10, 64)
    off, isc, val = T.lists()
    assert not isc.any()
    a = np.stack(T.force())
    b = np.stack(orc.direct_brute(x, y, z, m, 1.0, r_cut, eps))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.linalg.norm(b, axis=0))


def test_theta_error_trend(orc):
    """Sanity (no absolute pin exists): the tree error against the direct sum shrinks with
    theta roughly like theta^2 (Section 3.1.2), and the interaction count grows as theta
    falls (Section 3.2, N_int ~ theta^-2 at small theta)."""
    n, r_cut, eps = 20000, 0.06, 0.001
    x, y, z, m = boxgen.nfw_box(n, 30, 12)
    b = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, eps))
    nb = np.linalg.norm(b, axis=0)
    errs, ints = {}, {}
    for th in (0.25, 0.5, 1.0):
        T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, th, 10, 64)
        a = np.stack(T.force())
        errs[th] = np.sqrt(np.mean(np.linalg.norm(a - b, axis=0) ** 2)) / np.sqrt(np.mean(nb ** 2))
        ints[th] = T.interactions()
    assert errs[0.25] < errs[0.5] < errs[1.0]
    assert 1.5 < errs[0.5] / errs[0.25] < 16.0
    assert ints[0.25] > ints[0.5] > ints[1.0]


def test_lists_never_accept_a_node_holding_the_group(orc):
    """For theta > 1/sqrt(3) a node that contains the group can have its centre of mass far
    enough from the group's bbox to pass l < theta d; it must still be opened (the group's
    own particles cannot be replaced by a monopole that includes them).  Crafted box: a
    3-particle clump at the corner of the level-1 octant [0, 0.5)^3 whose mass sits in a
    100-particle clump at the opposite corner."""
    rng = boxgen.SplitMix64(21)
    small = 0.01 + 0.002 * rng.uniform(9).reshape(3, 3)
    big = 0.45 + 0.03 * rng.uniform(300).reshape(100, 3)
    far = 0.55 + 0.4 * rng.uniform(600).reshape(200, 3)
    pos = np.concatenate([small, big, far])
    m = np.full(pos.shape[0], 1.0 / pos.shape[0])
    for theta in (0.7, 1.0):
        T = orc.Tree(pos[:, 0], pos[:, 1], pos[:, 2], m, 1.0, 0.5, 0.001, theta, 2, 4)
        _frontier_check(orc, T, pos, m, theta, 0.5)
        # the octant [0, 0.5)^3 (code 0b1000) never appears as a cell entry of the small group
        G = T.groups()
        off, isc, val = T.lists()
        g0 = int(np.argmin(G["first"]))
        s, e = off[g0], off[g0 + 1]
        assert 8 not in [int(v) for v, c in zip(val[s:e], isc[s:e]) if c]


def test_opening_tie_opens_the_node(orc):
    """l = theta d exactly (dyadic positions, exact FP64) must open the node: the test is the
    strict l^2 < theta^2 d^2.  Group A = cube [0, 1/4)^3; node B = [1/4, 3/8) x [0, 1/8)^2
    holds two particles with centre of mass exactly 1/4 (= l / theta for l = 1/8,
    theta = 1/2) from A's bbox, so B itself is opened and its two children (side 1/16)
    are accepted instead."""
    pos = np.array([[0.03125, 0.03125, 0.03125], [0.0625, 0.0625, 0.0625],
                    [0.28125, 0.046875, 0.046875], [0.34375, 0.046875, 0.046875]])
    m = np.full(4, 0.25)
    T = orc.Tree(pos[:, 0], pos[:, 1], pos[:, 2], m, 1.0, 0.5, 0.001, 0.5, 2, 2)
    _frontier_check(orc, T, pos, m, 0.5, 0.5)
    G = T.groups()
    off, isc, val = T.lists()
    gA = int(np.argmin(G["first"]))
    cells = sorted(int(v) for v, c in zip(val[off[gA]:off[gA + 1]], isc[off[gA]:off[gA + 1]]) if c)
    # level-4 codes (marker 1 << 12) under B = level-3 code 0b1_000_100_000
    b3 = (1 << 9) | (0b000 << 6) | (0b100 << 3) | 0b000
    assert cells == sorted([(b3 << 3) | 0b000, (b3 << 3) | 0b100])


# ---------------------------------------------------------------- distance-dependent opening

# g_P3M of eq. (2) at R = 1/2, 1, 3/2, worked out by hand as exact fractions:
#   R = 1/2: 1 - (28 - 7 + 35/32 + 3/8 - 21/256)/140 = 1 - 5731/35840 = 30109/35840
#   R = 1  : 1 - (224 - 224 + 70 + 48 - 21)/140      = 43/140
#   R = 3/2: 1 - (12 - 504 + 3024 - 8505/2 + 1701 + 51030/64 - 6561/8 + 45927/256)/140
#          = 1 - 35103/35840 = 737/35840
G_EXACT = {0.5: 30109 / 35840, 1.0: 43 / 140, 1.5: 737 / 35840}


@pytest.mark.parametrize("eta", [1.0, 3.0 / 64.0, 0.001])
def test_theta_r_closed_forms(orc, eta):
    """theta(r) = theta_0 / sqrt(R g(R)), R = r / eta (eq. 12), below the cap."""
    for R, g in G_EXACT.items():
        for th0 in (0.01, 0.05, 0.2):
            want = th0 / math.sqrt(R * g)
            assert orc.theta_r(R * eta, eta, th0, 10.0) == pytest.approx(want, rel=1e-14)
    # the smallest angle sits where R g(R) peaks, near R = 0.65: theta >= theta_0 / 0.673
    rs = np.linspace(0.01, 1.99, 2000) * eta
    th = np.array([orc.theta_r(r, eta, 0.1, 10.0) for r in rs])
    assert 0.1 / math.sqrt(0.4528) < th.min() < 0.1 / math.sqrt(0.4526)
    assert 0.6 * eta < rs[np.argmin(th)] < 0.7 * eta


def test_theta_r_cap(orc):
    """The angle diverges at r -> 0 and r -> 2 eta (R g -> 0), so it is capped at theta_max;
    it equals theta_max exactly where R g(R) = 0 (r = 0, r >= r_cut)."""
    eta = 0.05
    for r in (0.0, 2 * eta, 3 * eta, 1.0):
        assert orc.theta_r(r, eta, 0.1, 0.7) == 0.7
    # near both ends the unlimited angle exceeds any cap
    assert orc.theta_r(1e-9, eta, 0.1, 0.7) == 0.7
    assert orc.theta_r(2 * eta * (1 - 1e-6), eta, 0.1, 0.7) == 0.7
    # in between it is below the cap and continuous across R = 1
    a, b = orc.theta_r(eta * (1 - 1e-9), eta, 0.1, 0.7), orc.theta_r(eta * (1 + 1e-9), eta,
                                                                    0.1, 0.7)
    assert a < 0.7 and b == pytest.approx(a, rel=1e-6)
    # a cap of 0 never accepts a node: the list force is the direct sum
    n, r_cut, eps = 3000, 0.1, 0.002
    x, y, z, m = boxgen.nfw_box(n, 20, 31)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.1, 10, 64, opening=1, theta_max=0.0)
    off, isc, val = T.lists()
    assert not isc.any()
    a = np.stack(T.force())
    b = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, eps))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.linalg.norm(b, axis=0))


@pytest.mark.parametrize("theta0,theta_max", [(0.05, 0.5), (0.15, 1.0), (0.3, 0.6)])
def test_distance_opening_lists_equal_brute_force_frontier(orc, theta0, theta_max):
    n, r_cut = 400, 0.2
    x, y, z, m = boxgen.nfw_box(n, 4, 5)
    T = orc.Tree(x, y, z, m, 1.0, r_cut, 0.003, theta0, 3, 20, opening=1, theta_max=theta_max)
    eta = 0.5 * r_cut
    _frontier_check(orc, T, np.stack([x, y, z], axis=1), m, theta0, r_cut,
                    theta_of_d=lambda d: orc.theta_r(d, eta, theta0, theta_max))


def test_distance_opening_reduces_to_fixed_at_the_cap(orc):
    """theta_0 so large that theta(r) >= theta_max everywhere: the lists are those of the
    fixed angle theta_max, entry for entry."""
    x, y, z, m = boxgen.nfw_box(3000, 20, 32)
    for tmax in (0.4, 0.8):
        F = orc.Tree(x, y, z, m, 1.0, 0.1, 0.002, tmax, 8, 48)
        V = orc.Tree(x, y, z, m, 1.0, 0.1, 0.002, 1.0e6, 8, 48, opening=1, theta_max=tmax)
        for a, b in zip(F.lists(), V.lists()):
            assert np.array_equal(a, b)


def test_distance_opening_beats_fixed_in_uniform_limit(orc):
    """Section 4.1: in the uniform-density limit a node's error scales as r theta^2 g(r/eta),
    so the angle of eq. (12) spreads the error evenly and should minimise it.  On the
    32^3 uniform box (r_cut = 3/32, eps = 1/640, n_crit = 64) theta_0 = 0.05 with cap 0.6
    costs fewer interactions than the fixed theta = 0.5 and has a several times smaller RMS
    relative error against the exact short-range force."""
    spec, (x, y, z, m) = boxgen.config_box("uniform32k")
    ex = np.stack(orc.direct_cells(x, y, z, m, spec.L, spec.r_cut, spec.eps), axis=1)
    mag = np.linalg.norm(ex, axis=1)

    def rms(T):
        a = np.stack(T.force(), axis=1)
        return float(np.sqrt(np.mean((np.linalg.norm(a - ex, axis=1) / mag) ** 2)))

    F = orc.Tree(x, y, z, m, spec.L, spec.r_cut, spec.eps, 0.5, spec.n_leaf, spec.n_crit)
    V = orc.Tree(x, y, z, m, spec.L, spec.r_cut, spec.eps, 0.05, spec.n_leaf, spec.n_crit,
                 opening=1, theta_max=0.6)
    assert V.interactions() < F.interactions()
    assert rms(V) < rms(F) / 4.0


# ---------------------------------------------------------------- quadrupole cells

def test_cutoff_derivatives(orc):
    """g' and g'' of eq. (2) used by the quadrupole term: against central differences of the
    (pinned) g itself on both branches, the known joins at R = 1 (g' = -1, g'' = 7/5) and zero
    from R = 2 on."""
    h, h2 = 1e-5, 1e-3   # the second difference needs the larger step (rounding / h^2)
    for R in list(np.linspace(0.05, 0.95, 19)) + list(np.linspace(1.05, 1.95, 19)):
        g1, g2 = orc.g_p3m_derivs(R)
        fd1 = (orc.g_p3m(R + h) - orc.g_p3m(R - h)) / (2 * h)
        fd2 = (orc.g_p3m(R + h2) - 2 * orc.g_p3m(R) + orc.g_p3m(R - h2)) / (h2 * h2)
        assert g1 == pytest.approx(fd1, rel=1e-7, abs=1e-9)
        assert g2 == pytest.approx(fd2, rel=0, abs=2e-5)
    for R in (1.0 - 1e-12, 1.0):
        g1, g2 = orc.g_p3m_derivs(R)
        assert g1 == pytest.approx(-1.0, abs=1e-9) and g2 == pytest.approx(1.4, abs=1e-9)
    assert orc.g_p3m_derivs(2.0) == (0.0, 0.0) and orc.g_p3m_derivs(3.0) == (0.0, 0.0)


def _cluster(s, seed=3):
    rng = np.random.default_rng(seed)
    offs = rng.standard_normal((3, 3))
    ms = np.array([0.5, 0.3, 0.2])
    offs -= (ms[:, None] * offs).sum(0) / ms.sum()
    pos = np.array([0.5, 0.5, 0.5]) + s * offs
    com = (ms[:, None] * pos).sum(0) / ms.sum()
    d = pos - com
    Q = np.array([(ms * d[:, a] * d[:, b]).sum() for a, b in
                  ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    return pos, ms, com, Q


@pytest.mark.parametrize("eps", [1e-4, 0.01])
@pytest.mark.parametrize("R", [0.3, 0.8, 1.2, 1.7])
def test_quadrupole_cell_is_third_order(orc, eps, R):
    """Section 4.1: the second-order term of a cell must carry the derivatives of the cutoff
    function.  Against the exact sum over a cell of three unequal masses (nonzero third
    moment), halving the cell's size divides the monopole's error by 4 (second order) and the
    quadrupole's by 8 (third order), on both branches of eq. (2) and with softening."""
    r_cut, L = 0.1, 1.0
    eta = r_cut / 2
    xi = np.array([0.5, 0.5, 0.5]) - R * eta * np.array([0.6, -0.48, 0.64])
    e1, e2 = [], []
    for s in (0.0005, 0.00025):
        pos, ms, com, Q = _cluster(s)
        ex = sum(orc.pair(xi, pos[j], ms[j], L, r_cut, eps) for j in range(3))
        e1.append(np.linalg.norm(orc.cell_acc(xi, com, ms.sum(), Q, L, r_cut, eps, 1) - ex))
        e2.append(np.linalg.norm(orc.cell_acc(xi, com, ms.sum(), Q, L, r_cut, eps, 2) - ex))
    assert 3.7 < e1[0] / e1[1] < 4.3
    assert 7.0 < e2[0] / e2[1] < 10.0
    assert e2[1] < 0.05 * e1[1]
    # beyond the cutoff the cell adds nothing, with or without the term
    far = np.array([0.5, 0.5, 0.5]) + np.array([2.05 * eta, 0.0, 0.0])
    pos, ms, com, Q = _cluster(0.0005)
    assert np.all(orc.cell_acc(far, com, ms.sum(), Q, L, r_cut, eps, 2) == 0.0)


def test_node_second_moments(orc):
    """Every node's second moment about its centre of mass equals the children's moments
    moved to it (parallel-axis theorem), is positive semi-definite, and its trace is
    sum m |x - com|^2 over the node's particles."""
    T, (x, y, z, m) = _tree(orc, 3000, 14, n_leaf=4, n_crit=24)
    nd = T.nodes()
    Q = T.nodes_q()
    k, idx = T.sorted()
    pos = np.stack([x, y, z], axis=1)[idx]
    ms = m[idx]
    codes = {int(c): u for u, c in enumerate(nd["code"])}
    full = lambda q: np.array([[q[0], q[3], q[4]], [q[3], q[1], q[5]], [q[4], q[5], q[2]]])
    for u in range(nd["code"].size):
        f, c = int(nd["first"][u]), int(nd["count"][u])
        d = pos[f:f + c] - nd["com"][u]
        tr = (ms[f:f + c] * (d * d).sum(axis=1)).sum()
        assert Q[u, :3].sum() == pytest.approx(tr, rel=1e-12, abs=1e-300)
        assert np.linalg.eigvalsh(full(Q[u])).min() >= -1e-12 * max(tr, 1e-300)
        if nd["nchild"][u]:
            code = int(nd["code"][u])
            kids = [codes[(code << 3) | o] for o in range(8) if (code << 3) | o in codes]
            S = np.zeros((3, 3))
            for v in kids:
                dv = nd["com"][v] - nd["com"][u]
                S += full(Q[v]) + nd["mass"][v] * np.outer(dv, dv)
            np.testing.assert_allclose(S, full(Q[u]), rtol=1e-10, atol=1e-14 * max(tr, 1e-300))


def test_quadrupole_tree_force_is_more_accurate(orc):
    """Section 4.1: the second-order term improves the accuracy a lot.  Same lists, theta =
    0.5, against the exact short-range sum of a clustered box: the 99th percentile of the
    relative error at least 5x smaller and the RMS (dominated by the few particles whose exact
    force nearly cancels) at least 1.8x smaller.  Measured here: p99 4.2e-2 -> 2.6e-3, RMS
    1.7e-2 -> 7.7e-3; on a 64^3 clustered box p99 5.0e-2 -> 3.4e-3, RMS 1.5e-2 -> 3.1e-3."""
    n, r_cut, eps = 20000, 0.06, 0.001
    x, y, z, m = boxgen.nfw_box(n, 30, 12)
    b = np.stack(orc.direct_cells(x, y, z, m, 1.0, r_cut, eps), axis=1)
    nb = np.linalg.norm(b, axis=1)
    err = {}
    for q in (False, True):
        T = orc.Tree(x, y, z, m, 1.0, r_cut, eps, 0.5, 10, 64, quadrupole=q)
        a = np.stack(T.force(), axis=1)
        e = np.linalg.norm(a - b, axis=1) / nb
        err[q] = (float(np.sqrt(np.mean(e ** 2))), float(np.quantile(e, 0.99)))
    assert err[True][0] < err[False][0] / 1.8
    assert err[True][1] < err[False][1] / 5.0


@pytest.mark.parametrize("opening,quad", [(0, False), (1, False), (0, True)],
                         ids=["fixed", "distance", "quadrupole"])
def test_walk_force_sample_equals_full_walk_and_force(orc, opening, quad):
    """The sampled walk + list force (the reference of the full-size parity tests and of the
    CPU baseline) against the whole-box walk, lists and list force: with stride 1 every
    particle's force and error scales equal the full computation bit for bit and the
    interaction count equals sum_g n_g L_g; with stride 7 and offset 3 exactly the particles
    of groups 3, 10, 17, ... are written, each equal to the full result, the others stay
    untouched, and the count is that of the sampled groups' lists."""
    x, y, z, m = boxgen.nfw_box(12000, 30, 77)
    T = orc.Tree(x, y, z, m, 1.0, 0.06, 0.001, 0.5, 10, 40, opening=opening,
                 theta_max=0.6 if opening else 0.0, quadrupole=quad)
    full = np.stack(T.force(nthreads=4))
    mag, newt = T.force_mag(nthreads=4)
    off, isc, val = T.lists()
    G = T.groups()
    lens = np.diff(off)
    ax, ay, az, inter, parts, ms, ns = T.walk_force_sample(1, 0, 4, scales=True)
    np.testing.assert_array_equal(np.stack([ax, ay, az]), full)
    np.testing.assert_array_equal(ms, mag)
    np.testing.assert_array_equal(ns, newt)
    assert inter == T.interactions() == int((G["count"] * lens).sum())
    assert parts == len(x)
    _, idx = T.sorted()
    sel = np.arange(3, T.n_groups, 7)
    want = np.zeros(len(x), dtype=bool)
    for g in sel:
        want[idx[G["first"][g]:G["first"][g] + G["count"][g]]] = True
    ax, ay, az, inter, parts, ms, ns = T.walk_force_sample(7, 3, 4, scales=True)
    got = np.stack([ax, ay, az])
    assert np.array_equal(~np.isnan(ax), want)
    np.testing.assert_array_equal(got[:, want], full[:, want])
    np.testing.assert_array_equal(ms[want], mag[want])
    np.testing.assert_array_equal(ns[want], newt[want])
    assert parts == int(want.sum()) == int(G["count"][sel].sum())
    assert inter == int((G["count"][sel] * lens[sel]).sum())
    # a new angle on the same tree gives the lists of a tree built with that angle
    T.set_theta(0.4)
    T2 = orc.Tree(x, y, z, m, 1.0, 0.06, 0.001, 0.4, 10, 40, opening=opening,
                  theta_max=0.6 if opening else 0.0, quadrupole=quad)
    for a, b in zip(T.lists(), T2.lists()):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(np.stack(T.force(nthreads=4)), np.stack(T2.force(nthreads=4)))
