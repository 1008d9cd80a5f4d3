"""Plain reference quadtree for the tree-code / multipole solve.

TEST INFRASTRUCTURE ONLY.  This is the bit-exact reference for the GPU tree
build: Morton keys, the stable target sort, the cells with their source and
target ranges, and the interaction lists.  It is written for clarity (Python
integers, recursion), not speed, and shares no code with the GPU library.

The paper groups sources hierarchically in a quadtree and treats a group as one
expanded source "at sufficiently large distances" (Appendix A, Multipole
Expansion, Fig. multipole and the superposition of group contributions).  It
does not say how the tree is built or what "sufficiently large" means; the
readings implemented here are:

* Root square: anchored at the grid origin (x0, y0) with side 2^k h, k the
  smallest integer with 2^k >= max(nx, ny).  The finest level D = k has cells
  of side h, so grid node (i, j) lies in finest cell (i, j).
* Morton key: bit b of the x index goes to key bit 2b, bit b of the y index to
  bit 2b+1.  A target's finest cell is q = floor((t - x0) / h) per axis (FP64
  subtraction then FP64 division); targets with q outside [0, 2^k) are outside
  the root.
* Sources: grid nodes with f != 0, in increasing key order.  Targets: stably
  sorted by key (ties keep input order).
* Cells: the root (level 0) always exists.  A cell at level l < D is split when
  it holds more than ``leaf_max`` sources or more than ``leaf_max`` targets;
  its children are visited in quadrant order q = qx + 2 qy and kept when they
  hold at least one source or target.  Cells are numbered level by level, in
  that order.
* Acceptance: target cell A and source cell B interact through expansions when
  (r_A + r_B) < theta * d, r the half-diagonal of a cell and d the distance of
  the centres.  It is decided exactly in integers: with theta = num/den and
  positions in units of half a finest cell, (S_A + S_B)^2 den^2 < 2 num^2 d^2
  (S = cell side).  theta is read as round(1000 theta) / 1000.
* Traversal (dual tree, target A against source B, starting at the roots):
  accepted -> M2L pair; else both leaves -> P2P pair; else A is a leaf -> B is
  split; else B is a leaf -> A is split; else both are split.  Only source
  cells with sources and target cells with targets are visited.
* The paper's own tree-code (a target sees each group either through its
  expansion or directly): per target leaf, a one-sided traversal of the source
  tree with the acceptance s_B / d < theta, d the distance from the leaf's
  square to B's centre (``bh_mac``, ``bh_lists``).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


def root_exponent(nx: int, ny: int) -> int:
    """Smallest k >= 0 with 2^k >= max(nx, ny)."""
    n = max(int(nx), int(ny))
    k = 0
    while (1 << k) < n:
        k += 1
    return k


def interleave(ix, iy) -> np.ndarray:
    """Morton key: x bit b -> key bit 2b, y bit b -> key bit 2b+1 (16 bits per axis)."""
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    key = np.zeros(np.broadcast(ix, iy).shape, dtype=np.uint64)
    for b in range(16):
        key |= ((ix >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((iy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def theta_rational(theta: float) -> tuple[int, int]:
    """theta as num/den in lowest terms, num = round(1000 theta), den = 1000."""
    num = int(round(theta * 1000.0))
    if not (1 <= num <= 999):
        raise ValueError("theta must lie in (0, 1)")
    g = math.gcd(num, 1000)
    return num // g, 1000 // g


def source_keys_grid(f: np.ndarray):
    """Keys and flat row-major indices of the nonzero grid nodes, in key order."""
    ny, nx = f.shape
    jj, ii = np.nonzero(f != 0.0)
    keys = interleave(ii, jj)
    order = np.argsort(keys, kind="stable")
    flat = (jj * nx + ii)[order]
    return keys[order], flat.astype(np.int64)


def target_cells(tx, ty, x0: float, y0: float, h: float, k: int):
    """Finest-level cell of each target: floor((t - x0) / h); raises if outside the root."""
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    qx = np.floor((tx - x0) / h)
    qy = np.floor((ty - y0) / h)
    lim = float(1 << k)
    if not (np.all(qx >= 0) and np.all(qx < lim) and np.all(qy >= 0) and np.all(qy < lim)):
        raise ValueError("target outside the root square")
    return qx.astype(np.int64), qy.astype(np.int64)


def target_keys_sorted(tx, ty, x0, y0, h, k):
    qx, qy = target_cells(tx, ty, x0, y0, h, k)
    keys = interleave(qx, qy)
    perm = np.argsort(keys, kind="stable")
    return keys[perm], perm.astype(np.int64)


@dataclasses.dataclass
class Tree:
    D: int
    level: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    sb: np.ndarray
    se: np.ndarray
    tb: np.ndarray
    te: np.ndarray
    leaf: np.ndarray
    child_begin: np.ndarray  # -1 for leaves
    nchild: np.ndarray
    parent: np.ndarray
    level_start: np.ndarray  # cells of level l are [level_start[l], level_start[l+1])

    @property
    def ncells(self) -> int:
        return int(self.level.size)

    def nsrc(self, c: int) -> int:
        return int(self.se[c] - self.sb[c])

    def ntgt(self, c: int) -> int:
        return int(self.te[c] - self.tb[c])

    def children(self, c: int):
        if self.child_begin[c] < 0:
            return range(0)
        return range(int(self.child_begin[c]), int(self.child_begin[c] + self.nchild[c]))


def build_tree(src_keys: np.ndarray, tgt_keys: np.ndarray, D: int, leaf_max: int) -> Tree:
    """Top-down construction from the sorted key arrays (finest level D)."""
    src_keys = np.asarray(src_keys, dtype=np.uint64)
    tgt_keys = np.asarray(tgt_keys, dtype=np.uint64)
    cells = [dict(level=0, ix=0, iy=0, sb=0, se=int(src_keys.size), tb=0, te=int(tgt_keys.size), parent=-1)]
    level_start = [0]
    cur = [0]
    lvl = 0
    while True:
        nxt = []
        for c in cur:
            cell = cells[c]
            split = lvl < D and ((cell["se"] - cell["sb"]) > leaf_max or (cell["te"] - cell["tb"]) > leaf_max)
            cell["leaf"] = not split
            cell["child_begin"] = -1
            cell["nchild"] = 0
            if not split:
                continue
            shift = np.uint64(2 * (D - lvl - 1))
            first = len(cells)
            for q in range(4):
                cx = 2 * cell["ix"] + (q & 1)
                cy = 2 * cell["iy"] + (q >> 1)
                prefix = int(interleave(cx, cy))
                lo = np.uint64(prefix) << shift
                hi = np.uint64(prefix + 1) << shift
                sb = int(np.searchsorted(src_keys, lo, side="left"))
                se = int(np.searchsorted(src_keys, hi, side="left"))
                tb = int(np.searchsorted(tgt_keys, lo, side="left"))
                te = int(np.searchsorted(tgt_keys, hi, side="left"))
                if se > sb or te > tb:
                    cells.append(dict(level=lvl + 1, ix=cx, iy=cy, sb=sb, se=se, tb=tb, te=te, parent=c))
                    nxt.append(len(cells) - 1)
            cell["child_begin"] = first
            cell["nchild"] = len(cells) - first
        if not nxt:
            break
        level_start.append(nxt[0])
        cur = nxt
        lvl += 1
    level_start.append(len(cells))

    def col(name, dtype=np.int64):
        return np.array([c[name] for c in cells], dtype=dtype)

    return Tree(D=D, level=col("level"), ix=col("ix"), iy=col("iy"), sb=col("sb"), se=col("se"), tb=col("tb"),
                te=col("te"), leaf=col("leaf", bool), child_begin=col("child_begin"), nchild=col("nchild"),
                parent=col("parent"), level_start=np.array(level_start, dtype=np.int64))


def mac(tree: Tree, a: int, b: int, num: int, den: int) -> bool:
    """Exact integer acceptance test for target cell a and source cell b."""
    D = tree.D
    la, lb = int(tree.level[a]), int(tree.level[b])
    ca_x = (2 * int(tree.ix[a]) + 1) << (D - la)
    ca_y = (2 * int(tree.iy[a]) + 1) << (D - la)
    cb_x = (2 * int(tree.ix[b]) + 1) << (D - lb)
    cb_y = (2 * int(tree.iy[b]) + 1) << (D - lb)
    sa = 1 << (D - la + 1)
    sb = 1 << (D - lb + 1)
    d2 = (ca_x - cb_x) ** 2 + (ca_y - cb_y) ** 2
    return (sa + sb) ** 2 * den * den < 2 * num * num * d2


def interaction_lists(tree: Tree, theta: float):
    """All (target cell, source cell) M2L pairs and P2P pairs of the dual traversal."""
    num, den = theta_rational(theta)
    m2l, p2p = [], []
    if tree.ncells == 0 or tree.nsrc(0) == 0 or tree.ntgt(0) == 0:
        return m2l, p2p

    def src_kids(b):
        return [c for c in tree.children(b) if tree.nsrc(c) > 0]

    def tgt_kids(a):
        return [c for c in tree.children(a) if tree.ntgt(c) > 0]

    stack = [(0, 0)]
    while stack:
        a, b = stack.pop()
        if mac(tree, a, b, num, den):
            m2l.append((a, b))
        elif tree.leaf[a] and tree.leaf[b]:
            p2p.append((a, b))
        elif tree.leaf[a]:
            stack.extend((a, bb) for bb in src_kids(b))
        elif tree.leaf[b]:
            stack.extend((aa, b) for aa in tgt_kids(a))
        else:
            stack.extend((aa, bb) for aa in tgt_kids(a) for bb in src_kids(b))
    return m2l, p2p


def lists_for_cell(tree: Tree, target: int, theta: float):
    """M2L and P2P source cells of one target cell (same traversal, restricted to its ancestors)."""
    num, den = theta_rational(theta)
    path = []
    c = target
    while c >= 0:
        path.append(c)
        c = int(tree.parent[c])
    on_path = set(path)
    m2l, p2p = [], []
    if tree.nsrc(0) == 0 or tree.ntgt(target) == 0:
        return m2l, p2p
    stack = [(0, 0)]
    while stack:
        a, b = stack.pop()
        if mac(tree, a, b, num, den):
            if a == target:
                m2l.append(b)
        elif tree.leaf[a] and tree.leaf[b]:
            if a == target:
                p2p.append(b)
        elif tree.leaf[a]:
            stack.extend((a, bb) for bb in tree.children(b) if tree.nsrc(bb) > 0)
        elif tree.leaf[b]:
            stack.extend((aa, b) for aa in tree.children(a) if aa in on_path)
        else:
            stack.extend((aa, bb) for aa in tree.children(a) if aa in on_path
                         for bb in tree.children(b) if tree.nsrc(bb) > 0)
    return sorted(m2l), sorted(p2p)


def bh_mac(tree: Tree, a: int, b: int, num: int, den: int) -> bool:
    """Acceptance of source cell b for every target of leaf a in the paper's tree-code
    (a group is expanded when it is far enough from the target; read here as s_b / d < theta,
    s_b the side of b and d the smallest distance from a's square to b's centre).  Exact in
    integers with positions in units of half a finest cell: s_b^2 den^2 < num^2 d^2."""
    D = tree.D
    la, lb = int(tree.level[a]), int(tree.level[b])
    ax0 = (2 * int(tree.ix[a])) << (D - la)
    ax1 = (2 * int(tree.ix[a]) + 2) << (D - la)
    ay0 = (2 * int(tree.iy[a])) << (D - la)
    ay1 = (2 * int(tree.iy[a]) + 2) << (D - la)
    cx = (2 * int(tree.ix[b]) + 1) << (D - lb)
    cy = (2 * int(tree.iy[b]) + 1) << (D - lb)
    dx = max(0, ax0 - cx, cx - ax1)
    dy = max(0, ay0 - cy, cy - ay1)
    sb = 1 << (D - lb + 1)
    return sb * sb * den * den < num * num * (dx * dx + dy * dy)


def bh_lists(tree: Tree, theta: float):
    """Per target leaf a (leaves holding targets): the source cells whose multipoles are
    evaluated at a's targets (M2P) and the source leaves summed directly (P2P), from a
    traversal of the source tree that starts at the root: accepted -> M2P; a leaf -> P2P;
    otherwise its children with sources are visited.  Returns {a: (m2p, p2p)}, sorted."""
    num, den = theta_rational(theta)
    out = {}
    for a in range(tree.ncells):
        if not tree.leaf[a] or tree.ntgt(a) == 0:
            continue
        m2p, p2p = [], []
        stack = [0] if tree.nsrc(0) > 0 else []
        while stack:
            b = stack.pop()
            if bh_mac(tree, a, b, num, den):
                m2p.append(b)
            elif tree.leaf[b]:
                p2p.append(b)
            else:
                stack.extend(c for c in tree.children(b) if tree.nsrc(c) > 0)
        out[a] = (sorted(m2p), sorted(p2p))
    return out


def grid_tree(f: np.ndarray, tx, ty, h: float, x0: float = 0.0, y0: float = 0.0, leaf_max: int = 64):
    """Keys, permutations and tree for grid sources f[j, i] and the given targets."""
    ny, nx = f.shape
    k = root_exponent(nx, ny)
    skeys, sflat = source_keys_grid(f)
    tkeys, tperm = target_keys_sorted(tx, ty, x0, y0, h, k)
    tree = build_tree(skeys, tkeys, k, leaf_max)
    return dict(k=k, src_keys=skeys, src_flat=sflat, tgt_keys=tkeys, tgt_perm=tperm, tree=tree)
