"""Pins of the CPU near-field references used by the Kahan test (no GPU).

With one leaf holding every source and target, the near field of a target is
the whole direct sum, so the FP64 reference must equal 2 pi times the oracle's
P (plus ln(h) w for a coincident node, the library's convention for the
partial sums), and the uncompensated FP32 sum must agree with it to FP32
rounding.  With many leaves, the near sums of a leaf's targets plus the
oracle's direct sum over the sources outside its near list is the full sum.
"""

import math

import numpy as np

from oracle import direct, tree_ref

from near_emulation import near_lists, near_sums


def _case(n=24, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.standard_normal((n, n))
    f[rng.uniform(size=f.shape) < 0.2] = 0.0
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    tx = np.concatenate([rng.uniform(0, 1, 200), xs[[2, 7, 11]]])
    ty = np.concatenate([rng.uniform(0, 1, 200), xs[[5, 0, 23]]])
    return f, h, tx, ty


def test_single_leaf_is_the_direct_sum():
    f, h, tx, ty = _case()
    info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=10**6)
    assert info["tree"].ncells == 1
    lists = near_lists(info["tree"], 0.5)
    ref, naive, idx = near_sums(f, h, tx, ty, info, lists, [0])
    perm = info["tgt_perm"][idx]
    P = direct.direct_grid(f, h, tx[perm], ty[perm])
    # coincident nodes: the partial sums carry ln(h) w of the node
    ii = np.floor(tx[perm] / h).astype(int)
    jj = np.floor(ty[perm] / h).astype(int)
    on = (tx[perm] == (ii + 0.5) * h) & (ty[perm] == (jj + 0.5) * h)
    wself = np.where(on, f[jj, ii] * h * h, 0.0)
    expect = 2 * math.pi * P + math.log(h) * wself
    assert on.sum() == 3
    np.testing.assert_allclose(ref, expect, rtol=1e-12, atol=1e-13 * np.abs(expect).max())
    assert np.max(np.abs(naive - expect)) < 1e-5 * np.abs(expect).max()


def test_near_plus_rest_is_the_direct_sum():
    f, h, tx, ty = _case(n=32, seed=4)
    info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=8)
    t = info["tree"]
    lists = near_lists(t, 0.5)
    leaves = sorted(lists)[:6]
    ref, _, idx = near_sums(f, h, tx, ty, info, lists, leaves)
    flat = info["src_flat"]
    perm = info["tgt_perm"]
    pos = 0
    for A in leaves:
        inside = np.zeros(flat.size, bool)
        for B in lists[A]:
            inside[t.sb[B]:t.se[B]] = True
        g = np.zeros_like(f)
        g.ravel()[flat[~inside]] = f.ravel()[flat[~inside]]
        k = idx[pos:pos + (t.te[A] - t.tb[A])]
        kx, ky = tx[perm[k]], ty[perm[k]]
        rest = 2 * math.pi * direct.direct_grid(g, h, kx, ky)
        full = 2 * math.pi * direct.direct_grid(f, h, kx, ky)
        ii = np.floor(kx / h).astype(int)
        jj = np.floor(ky / h).astype(int)
        on = (kx == (ii + 0.5) * h) & (ky == (jj + 0.5) * h)
        full += math.log(h) * np.where(on, f[jj, ii] * h * h, 0.0)
        np.testing.assert_allclose(ref[pos:pos + k.size] + rest, full, rtol=1e-11, atol=1e-12 * np.abs(full).max())
        pos += k.size
