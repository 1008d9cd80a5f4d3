"""Pins of the reference quadtree (Morton keys, sort, cells, interaction lists).

The paper groups sources in a hierarchical quadtree and evaluates far groups
through expansions and the rest directly, summing the group contributions
(Appendix A, Fig. multipole and the superposition equation that follows it).
The pins: hand-computed Morton keys, sort stability, the cell invariants, and
the counting invariant (every target/source pair is covered by exactly one
interaction), checked by brute force.
"""

import numpy as np
import pytest

from oracle import tree_ref
from workloads import generators as G


def test_interleave_hand_values():
    assert int(tree_ref.interleave(0, 0)) == 0
    assert int(tree_ref.interleave(1, 0)) == 1
    assert int(tree_ref.interleave(0, 1)) == 2
    assert int(tree_ref.interleave(3, 3)) == 15
    # x = 0b101, y = 0b110 -> bits (y2 x2 y1 x1 y0 x0) = 1 1 1 0 0 1 = 0b111001
    assert int(tree_ref.interleave(5, 6)) == 0b111001
    assert int(tree_ref.interleave(0xFFFF, 0)) == 0x55555555
    assert int(tree_ref.interleave(0, 0xFFFF)) == 0xAAAAAAAA


def test_root_exponent_and_theta():
    assert tree_ref.root_exponent(1, 1) == 0
    assert tree_ref.root_exponent(64, 64) == 6
    assert tree_ref.root_exponent(65, 3) == 7
    assert tree_ref.theta_rational(0.5) == (1, 2)
    assert tree_ref.theta_rational(0.4) == (2, 5)
    with pytest.raises(ValueError):
        tree_ref.theta_rational(1.0)


def test_target_sort_is_stable():
    tx = np.array([0.9, 0.1, 0.12, 0.9, 0.11])
    ty = np.array([0.9, 0.1, 0.1, 0.9, 0.1])
    keys, perm = tree_ref.target_keys_sorted(tx, ty, 0.0, 0.0, 0.25, 2)
    # cells: (3,3), (0,0), (0,0), (3,3), (0,0)
    assert list(perm) == [1, 2, 4, 0, 3]
    assert list(keys) == [0, 0, 0, 15, 15]


def test_target_outside_root_raises():
    with pytest.raises(ValueError):
        tree_ref.target_keys_sorted([1.0], [0.5], 0.0, 0.0, 0.25, 2)
    with pytest.raises(ValueError):
        tree_ref.target_keys_sorted([-1e-12], [0.5], 0.0, 0.0, 0.25, 2)


def _small_case(seed=1, n=32, nt=300, leaf_max=8, zero_frac=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.standard_normal((n, n))
    f[rng.uniform(size=f.shape) < zero_frac] = 0.0
    h = 1.0 / n
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    # targets: some nodes, a cluster, uniform points
    tx = np.concatenate([x.ravel()[::5], 0.3 + 0.01 * rng.standard_normal(nt // 3), rng.uniform(0, 1, nt)])
    ty = np.concatenate([y.ravel()[::5], 0.7 + 0.01 * rng.standard_normal(nt // 3), rng.uniform(0, 1, nt)])
    info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=leaf_max)
    return f, tx, ty, info


def test_cell_invariants():
    f, tx, ty, info = _small_case()
    t = info["tree"]
    D = t.D
    assert t.sb[0] == 0 and t.se[0] == info["src_keys"].size and t.te[0] == tx.size
    leaf_src = np.zeros(info["src_keys"].size, int)
    leaf_tgt = np.zeros(tx.size, int)
    for c in range(t.ncells):
        assert t.nsrc(c) + t.ntgt(c) > 0 or c == 0
        if t.leaf[c]:
            leaf_src[t.sb[c]:t.se[c]] += 1
            leaf_tgt[t.tb[c]:t.te[c]] += 1
            assert t.level[c] == D or (t.nsrc(c) <= 8 and t.ntgt(c) <= 8)
        else:
            kids = list(t.children(c))
            assert 1 <= len(kids) <= 4
            assert sum(t.nsrc(k) for k in kids) == t.nsrc(c)
            assert sum(t.ntgt(k) for k in kids) == t.ntgt(c)
            for k in kids:
                assert t.parent[k] == c and t.level[k] == t.level[c] + 1
                assert t.ix[k] // 2 == t.ix[c] and t.iy[k] // 2 == t.iy[c]
        # every key in the cell's ranges has the cell's prefix
        sh = np.uint64(2 * (D - t.level[c]))
        pre = tree_ref.interleave(t.ix[c], t.iy[c])
        assert np.all((info["src_keys"][t.sb[c]:t.se[c]] >> sh) == pre)
        assert np.all((info["tgt_keys"][t.tb[c]:t.te[c]] >> sh) == pre)
    assert np.all(leaf_src == 1) and np.all(leaf_tgt == 1)


def test_counting_invariant_brute_force():
    """Every (target, source) pair is covered exactly once by the M2L and P2P lists."""
    for seed, lm in ((1, 8), (2, 4), (3, 16)):
        f, tx, ty, info = _small_case(seed=seed, leaf_max=lm)
        t = info["tree"]
        m2l, p2p = tree_ref.interaction_lists(t, 0.5)
        ns, nt = info["src_keys"].size, tx.size
        cover = np.zeros((nt, ns), dtype=np.int32)
        for a, b in m2l + p2p:
            cover[t.tb[a]:t.te[a], t.sb[b]:t.se[b]] += 1
        assert np.all(cover == 1)
        # and every P2P pair is between leaves, every M2L pair is accepted
        for a, b in p2p:
            assert t.leaf[a] and t.leaf[b]
        num, den = tree_ref.theta_rational(0.5)
        for a, b in m2l:
            assert tree_ref.mac(t, a, b, num, den)


def test_mac_matches_geometry():
    """The integer test equals (r_A + r_B) < theta d in exact arithmetic (checked with fractions)."""
    from fractions import Fraction
    f, tx, ty, info = _small_case(seed=4)
    t = info["tree"]
    rng = np.random.Generator(np.random.PCG64(0))
    for _ in range(400):
        a, b = rng.integers(0, t.ncells, 2)
        for theta, (num, den) in ((0.5, (1, 2)), (0.4, (2, 5))):
            sa = Fraction(1, 2 ** int(t.level[a]))
            sb = Fraction(1, 2 ** int(t.level[b]))
            cax = (t.ix[a] + Fraction(1, 2)) * sa
            cay = (t.iy[a] + Fraction(1, 2)) * sa
            cbx = (t.ix[b] + Fraction(1, 2)) * sb
            cby = (t.iy[b] + Fraction(1, 2)) * sb
            d2 = (cax - cbx) ** 2 + (cay - cby) ** 2
            # (sa+sb)/sqrt2 < theta d  <=>  (sa+sb)^2 < 2 theta^2 d^2
            geo = (sa + sb) ** 2 < 2 * Fraction(num, den) ** 2 * d2
            assert geo == tree_ref.mac(t, int(a), int(b), num, den)


def test_lists_for_cell_agree_with_full_traversal():
    f, tx, ty, info = _small_case(seed=5, leaf_max=6)
    t = info["tree"]
    m2l, p2p = tree_ref.interaction_lists(t, 0.4)
    for a in range(t.ncells):
        if t.ntgt(a) == 0:
            continue
        lm, lp = tree_ref.lists_for_cell(t, a, 0.4)
        assert lm == sorted(b for aa, b in m2l if aa == a)
        assert lp == sorted(b for aa, b in p2p if aa == a)


def test_uniform_grid_counts():
    """64^2 uniform grid, targets = nodes, leaf 8x8 (leaf_max 64), theta 0.5: a uniform depth-3 tree."""
    g = G.GridSpec(64, 64, 1.0 / 64)
    f = G.gaussian_source(g)
    x, y = G.grid_nodes(g)
    info = tree_ref.grid_tree(f, x.ravel(), y.ravel(), g.h, leaf_max=64)
    t = info["tree"]
    assert t.ncells == 1 + 4 + 16 + 64
    assert np.all(t.leaf == (t.level == 3))
    m2l, p2p = tree_ref.interaction_lists(t, 0.5)
    # every leaf's P2P neighbourhood is a block of leaves around it; totals from the traversal
    assert len(p2p) == 1156 and len(m2l) == 2040


def test_bh_mac_matches_geometry():
    """The tree-code test s_B / d < theta (d from the leaf's square to B's centre) in exact arithmetic."""
    from fractions import Fraction
    f, tx, ty, info = _small_case(seed=6, leaf_max=4)
    t = info["tree"]
    rng = np.random.Generator(np.random.PCG64(1))
    leaves = [a for a in range(t.ncells) if t.leaf[a]]
    for _ in range(400):
        a = int(rng.choice(leaves))
        b = int(rng.integers(0, t.ncells))
        for theta, (num, den) in ((0.5, (1, 2)), (0.4, (2, 5)), (0.7, (7, 10))):
            sa = Fraction(1, 2 ** int(t.level[a]))
            sb = Fraction(1, 2 ** int(t.level[b]))
            x0, x1 = t.ix[a] * sa, (t.ix[a] + 1) * sa
            y0, y1 = t.iy[a] * sa, (t.iy[a] + 1) * sa
            cbx = (t.ix[b] + Fraction(1, 2)) * sb
            cby = (t.iy[b] + Fraction(1, 2)) * sb
            dx = max(Fraction(0), x0 - cbx, cbx - x1)
            dy = max(Fraction(0), y0 - cby, cby - y1)
            geo = sb ** 2 < Fraction(num, den) ** 2 * (dx * dx + dy * dy)
            assert geo == tree_ref.bh_mac(t, a, b, num, den)


def test_bh_lists_cover_every_pair_once():
    """Per target leaf, the accepted cells and the direct leaves partition the sources exactly once;
    accepted cells lie outside the leaf, direct cells are leaves."""
    for seed, lm, theta in ((1, 8, 0.5), (2, 4, 0.4), (3, 16, 0.6)):
        f, tx, ty, info = _small_case(seed=seed, leaf_max=lm)
        t = info["tree"]
        ns = info["src_keys"].size
        num, den = tree_ref.theta_rational(theta)
        lists = tree_ref.bh_lists(t, theta)
        assert set(lists) == {a for a in range(t.ncells) if t.leaf[a] and t.ntgt(a) > 0}
        for a, (m2p, p2p) in lists.items():
            cover = np.zeros(ns, dtype=np.int32)
            for b in m2p + p2p:
                cover[t.sb[b]:t.se[b]] += 1
            assert np.all(cover == 1), a
            for b in m2p:
                assert tree_ref.bh_mac(t, a, b, num, den)
                # B's square and A's square are disjoint (the target never sits inside an accepted group)
                la, lb = int(t.level[a]), int(t.level[b])
                lo = min(la, lb)
                assert not (t.ix[a] >> (la - lo) == t.ix[b] >> (lb - lo)
                            and t.iy[a] >> (la - lo) == t.iy[b] >> (lb - lo)), (a, b)
            assert all(t.leaf[b] for b in p2p)
