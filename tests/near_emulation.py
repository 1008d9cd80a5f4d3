"""CPU references for the near field of sampled target leaves (Kahan pin).

TEST INFRASTRUCTURE.  The tree and the near (P2P) lists come from the
reference quadtree (``oracle.tree_ref``), never from the GPU library.  For each
target of the sampled leaves this computes

* ``ref``:   the near field sum_{near sources s != t} w_s ln|t - s| in FP64,
             plus ln(h) w for a coincident node (the library's near partial
             sums carry that term; the finalize step removes it), and
* ``naive``: the same sum evaluated the way a plain FP32 kernel would, with
             FP32 offsets in units of h from the leaf corners, FP32 weights,
             log2 of the FP32 squared distance, and an uncompensated FP32
             running sum per list part (the parts split a leaf's list the way
             the library does: entries [k nb / parts, (k + 1) nb / parts)).

Appendix A, eq. greenSum restricted to the non-accepted leaf pairs.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import tree_ref


def near_lists(tree, theta):
    """P2P source leaves of every target leaf (reference lists, sorted)."""
    _, p2p = tree_ref.interaction_lists(tree, theta)
    out = {}
    for a, b in p2p:
        out.setdefault(int(a), []).append(int(b))
    return {a: sorted(v) for a, v in out.items()}


def near_sums(f, h, tx, ty, info, lists, leaves, nparts=5):
    """(ref, naive, target index in sorted order) for every target of `leaves`."""
    t = info["tree"]
    D = t.D
    ny, nx = f.shape
    flat = info["src_flat"]
    si = flat % nx
    sj = flat // nx
    wsrc = f.ravel()[flat] * h * h
    perm = info["tgt_perm"]
    TX = np.asarray(tx, dtype=np.float64)[perm]
    TY = np.asarray(ty, dtype=np.float64)[perm]
    f32 = np.float32
    lnh = math.log(h)
    refs, naives, idx = [], [], []
    for A in leaves:
        shA = D - int(t.level[A])
        cax = int(t.ix[A]) << shA
        cay = int(t.iy[A]) << shA
        tb, te = int(t.tb[A]), int(t.te[A])
        relx = TX[tb:te] / h - cax
        rely = TY[tb:te] / h - cay
        rx32 = relx.astype(f32)
        ry32 = rely.astype(f32)
        Bs = lists.get(A, [])
        nb = len(Bs)
        ref = np.zeros(te - tb)
        naive = np.zeros(te - tb)
        for part in range(nparts):
            e0 = part * nb // nparts
            e1 = (part + 1) * nb // nparts
            run = np.zeros(te - tb, f32)
            wn = 0.0
            for B in Bs[e0:e1]:
                shB = D - int(t.level[B])
                cbx = int(t.ix[B]) << shB
                cby = int(t.iy[B]) << shB
                s0, s1 = int(t.sb[B]), int(t.se[B])
                ox = si[s0:s1] + 0.5 - cbx
                oy = sj[s0:s1] + 0.5 - cby
                ws = wsrc[s0:s1]
                wn += float(ws.sum())
                # FP64: exact half-integer source offsets, FP64 target offsets
                dx = (relx + (cax - cbx))[:, None] - ox[None, :]
                dy = (rely + (cay - cby))[:, None] - oy[None, :]
                r2 = dx * dx + dy * dy
                with np.errstate(divide="ignore"):
                    lg = np.where(r2 > 0.0, np.log(np.where(r2 > 0.0, r2, 1.0)), 0.0)
                ref += 0.5 * (lg * ws[None, :]).sum(axis=1)
                # FP32, uncompensated, sources in order
                tx32 = (rx32 + f32(cax - cbx)).astype(f32)
                ty32 = (ry32 + f32(cay - cby)).astype(f32)
                dx32 = (tx32[:, None] - ox.astype(f32)[None, :]).astype(f32)
                dy32 = (ty32[:, None] - oy.astype(f32)[None, :]).astype(f32)
                r232 = (dx32 * dx32 + dy32 * dy32).astype(f32)
                r232 = np.where(r232 == 0.0, f32(1.0), r232)
                terms = (ws.astype(f32)[None, :] * np.log2(r232)).astype(f32)
                for i in range(s1 - s0):
                    run = (run + terms[:, i]).astype(f32)
            ref += lnh * wn
            naive += 0.5 * (run.astype(np.float64) * math.log(2.0)) + lnh * wn
        refs.append(ref)
        naives.append(naive)
        idx.append(np.arange(tb, te))
    return np.concatenate(refs), np.concatenate(naives), np.concatenate(idx)
