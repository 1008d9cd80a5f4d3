"""Plain FP64 expansion operators and a slow reference tree-code/FMM.

TEST INFRASTRUCTURE ONLY.  Written in the paper's notation (Appendix A,
Multipole Expansion): a group of sources w_i = f_i h_i^2 at z_i, expanded about
a centre z_c, is

    S = sum_i w_i,   alpha_k = sum_i w_i (z_i - z_c)^k / k,            (eq. alphaK)
    P(z) = (1/2pi) [ S Re log(z - z_c) - sum_k Re alpha_k / (z - z_c)^k ]   (eq. pressTruncated)

Readings of the printed equations (each checked by a test):
* eq. pressTruncated prints the 1/2pi factor on the S term only; eq. expanded1,
  from which it is derived, has it on both terms, so both carry it here.
* eq. expandedBeta prints the S term of the shifted coefficient with a minus
  sign; expanding S log(z - z_c) about z_p with eq. logExpansion gives
  beta_k = + S z0^k / k + sum_{l<=k} alpha_l z0^{k-l} C(k-1, l-1), z0 = z_c - z_p,
  which is what ``m2m`` implements (the exactness test fails with the printed sign).

The local-expansion operators (M2L, L2L, L2P) come from the fast multipole
method the paper cites for the O(N) variant; they follow from eq. logExpansion
applied with the roles of z and z' exchanged:

    M2L: with z0 = z_B - z_A (source centre minus target centre)
        L_0 = S log|z0| - sum_k alpha_k (-z0)^{-k}     (real part is all that is kept of log)
        L_l = -S / (l z0^l) - z0^{-l} sum_k alpha_k (-z0)^{-k} C(l+k-1, k-1),  l >= 1
    L2L: L'_m = sum_{l>=m} L_l C(l, m) d^{l-m},  d = z_child - z_parent
    L2P: P(z) += (1/2pi) Re sum_l L_l (z - z_A)^l

The paper's own tree-code (``treecode_grid``) uses no local expansions: each
target leaf evaluates the multipole of every accepted group at its targets
(M2P, eq. pressTruncated) and sums the other leaves directly; acceptance is
``tree_ref.bh_mac``.

All arrays are complex128; nothing is scaled.
"""

from __future__ import annotations

import math

import numpy as np

from . import tree_ref

TWO_PI = 2.0 * math.pi


def binom(n: int, k: int) -> float:
    return float(math.comb(n, k)) if 0 <= k <= n else 0.0


def p2m(z, w, zc, p: int):
    """(S, alpha[1..p]) of sources z (complex) with weights w about zc. alpha[0] is unused (0)."""
    z = np.asarray(z, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    S = float(np.sum(w))
    alpha = np.zeros(p + 1, dtype=np.complex128)
    d = z - zc
    for k in range(1, p + 1):
        alpha[k] = np.sum(w * d**k) / k
    return S, alpha


def m2p(S, alpha, zc, z):
    """P(z) of one expansion, eq. pressTruncated (both terms carry 1/2pi)."""
    z = np.asarray(z, dtype=np.complex128)
    u = z - zc
    acc = S * np.log(np.abs(u))
    for k in range(1, alpha.size):
        acc = acc - np.real(alpha[k] / u**k)
    return acc / TWO_PI


def m2m(S, alpha, z_child, z_parent):
    """Shift a child expansion to its parent's centre (corrected eq. expandedBeta)."""
    p = alpha.size - 1
    z0 = complex(z_child) - complex(z_parent)
    beta = np.zeros(p + 1, dtype=np.complex128)
    for k in range(1, p + 1):
        acc = S * z0**k / k
        for l in range(1, k + 1):
            acc += alpha[l] * z0 ** (k - l) * binom(k - 1, l - 1)
        beta[k] = acc
    return S, beta


def m2l(S, alpha, z_src, z_tgt, p: int):
    """Local coefficients L[0..p] at z_tgt of the expansion (S, alpha) about z_src."""
    z0 = complex(z_src) - complex(z_tgt)
    L = np.zeros(p + 1, dtype=np.complex128)
    q = alpha.size - 1
    L[0] = S * math.log(abs(z0)) - sum(alpha[k] * (-z0) ** (-k) for k in range(1, q + 1))
    for l in range(1, p + 1):
        acc = -S / (l * z0**l)
        for k in range(1, q + 1):
            acc -= alpha[k] * (-z0) ** (-k) * binom(l + k - 1, k - 1) * z0 ** (-l)
        L[l] = acc
    return L


def l2l(L, z_parent, z_child):
    """Re-centre a local expansion from z_parent to z_child (exact for a polynomial)."""
    p = L.size - 1
    d = complex(z_child) - complex(z_parent)
    out = np.zeros(p + 1, dtype=np.complex128)
    for m in range(p + 1):
        out[m] = sum(L[l] * binom(l, m) * d ** (l - m) for l in range(m, p + 1))
    return out


def l2p(L, zc, z):
    """(1/2pi) Re sum_l L_l (z - zc)^l."""
    u = np.asarray(z, dtype=np.complex128) - zc
    acc = np.zeros(u.shape, dtype=np.complex128)
    for l in range(L.size - 1, -1, -1):
        acc = acc * u + L[l]
    return np.real(acc) / TWO_PI


def _upward(tree, zs, ws, centre, p: int):
    """P2M at the source leaves, then M2M from the finest level up (unscaled S, alpha per cell)."""
    nc = tree.ncells
    S = np.zeros(nc)
    alpha = np.zeros((nc, p + 1), dtype=np.complex128)
    for c in range(nc - 1, -1, -1):
        if tree.nsrc(c) == 0:
            continue
        if tree.leaf[c]:
            sl = slice(int(tree.sb[c]), int(tree.se[c]))
            S[c], alpha[c] = p2m(zs[sl], ws[sl], centre(c), p)
        else:
            for ch in tree.children(c):
                if tree.nsrc(ch) == 0:
                    continue
                s2, b = m2m(S[ch], alpha[ch], centre(ch), centre(c))
                S[c] += s2
                alpha[c] += b
    return S, alpha


def _near(tree, pairs, txs, tys, sxs, sys_, ws, h, self_mode, near):
    """Direct sum over (target leaf, source leaf) pairs into near[sorted target], without 1/2pi;
    coincident pairs skipped (or replaced by the cell average)."""
    lnh = math.log(h)
    kappa = 1.5 - math.pi / 4.0 + 0.5 * math.log(2.0)
    for a, b in pairs:
        tl = range(int(tree.tb[a]), int(tree.te[a]))
        sl = slice(int(tree.sb[b]), int(tree.se[b]))
        for t in tl:
            dx = txs[t] - sxs[sl]
            dy = tys[t] - sys_[sl]
            r2 = dx * dx + dy * dy
            self_ = r2 == 0.0
            contrib = np.where(self_, 0.0, ws[sl] * 0.5 * np.log(np.where(self_, 1.0, r2)))
            near[t] += float(np.sum(contrib))
            if self_mode == 1 and np.any(self_):
                near[t] += float(np.sum(ws[sl][self_])) * (lnh - kappa)
    near /= TWO_PI


def fmm_grid(f, tx, ty, h, p: int, theta: float, leaf_max: int = 64, x0: float = 0.0, y0: float = 0.0,
             self_mode: int = 0):
    """Slow reference tree-code (P2M, M2M, M2L, L2L, L2P, P2P) on grid sources.

    Returns dict(P=..., far=..., near=..., S=..., alpha=..., L=..., tree=...): P and its far
    (L2P) and near (P2P) parts in the caller's target order, each including the 1/2pi factor,
    plus the per-cell multipoles (S, alpha) and locals L (without 1/2pi).
    """
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    info = tree_ref.grid_tree(f, tx, ty, h, x0, y0, leaf_max)
    tree = info["tree"]
    k = info["k"]
    m2l_pairs, p2p_pairs = tree_ref.interaction_lists(tree, theta)
    flat = info["src_flat"]
    si = flat % nx
    sj = flat // nx
    sxs = x0 + (si + 0.5) * h
    sys_ = y0 + (sj + 0.5) * h
    zs = sxs + 1j * sys_
    ws = f.ravel()[flat] * h * h
    perm = info["tgt_perm"]
    txs, tys = tx[perm], ty[perm]
    zt = txs + 1j * tys
    nc = tree.ncells

    def centre(c):
        side = h * 2.0 ** (k - int(tree.level[c]))
        return complex(x0 + (int(tree.ix[c]) + 0.5) * side, y0 + (int(tree.iy[c]) + 0.5) * side)

    S, alpha = _upward(tree, zs, ws, centre, p)
    # downward pass
    L = np.zeros((nc, p + 1), dtype=np.complex128)
    for a, b in m2l_pairs:
        L[a] += m2l(S[b], alpha[b], centre(b), centre(a), p)
    for c in range(nc):
        par = int(tree.parent[c])
        if par >= 0 and tree.ntgt(c) > 0:
            L[c] += l2l(L[par], centre(par), centre(c))
    far = np.zeros(tx.size)
    near = np.zeros(tx.size)
    for c in range(nc):
        if not tree.leaf[c] or tree.ntgt(c) == 0:
            continue
        tl = slice(int(tree.tb[c]), int(tree.te[c]))
        far[tl] = l2p(L[c], centre(c), zt[tl])
    _near(tree, p2p_pairs, txs, tys, sxs, sys_, ws, h, self_mode, near)
    out_far = np.empty_like(far)
    out_near = np.empty_like(near)
    out_far[perm] = far
    out_near[perm] = near
    return dict(P=out_far + out_near, far=out_far, near=out_near, S=S, alpha=alpha, L=L, tree=tree,
                info=info, m2l=m2l_pairs, p2p=p2p_pairs)


def treecode_grid(f, tx, ty, h, p: int, theta: float, leaf_max: int = 64, x0: float = 0.0, y0: float = 0.0,
                  self_mode: int = 0):
    """Slow reference of the paper's own tree-code on grid sources: P2M and M2M upward, then
    for every target leaf the multipoles of the accepted cells evaluated at its targets
    (eq. pressTruncated, M2P) and a direct sum over the other leaves (``tree_ref.bh_lists``).
    Returns dict(P, far, near, S, alpha, tree, lists) in the caller's target order (1/2pi included).
    """
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    info = tree_ref.grid_tree(f, tx, ty, h, x0, y0, leaf_max)
    tree = info["tree"]
    k = info["k"]
    lists = tree_ref.bh_lists(tree, theta)
    flat = info["src_flat"]
    sxs = x0 + (flat % nx + 0.5) * h
    sys_ = y0 + (flat // nx + 0.5) * h
    ws = f.ravel()[flat] * h * h
    perm = info["tgt_perm"]
    txs, tys = tx[perm], ty[perm]
    zt = txs + 1j * tys

    def centre(c):
        side = h * 2.0 ** (k - int(tree.level[c]))
        return complex(x0 + (int(tree.ix[c]) + 0.5) * side, y0 + (int(tree.iy[c]) + 0.5) * side)

    S, alpha = _upward(tree, sxs + 1j * sys_, ws, centre, p)
    far = np.zeros(tx.size)
    near = np.zeros(tx.size)
    pairs = []
    for a, (m2p_cells, p2p_cells) in lists.items():
        tl = slice(int(tree.tb[a]), int(tree.te[a]))
        for b in m2p_cells:
            far[tl] += m2p(S[b], alpha[b], centre(b), zt[tl])
        pairs.extend((a, b) for b in p2p_cells)
    _near(tree, pairs, txs, tys, sxs, sys_, ws, h, self_mode, near)
    out_far = np.empty_like(far)
    out_near = np.empty_like(near)
    out_far[perm] = far
    out_near[perm] = near
    return dict(P=out_far + out_near, far=out_far, near=out_near, S=S, alpha=alpha, tree=tree, info=info,
                lists=lists)
