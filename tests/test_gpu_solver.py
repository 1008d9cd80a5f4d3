"""GPU parity of the HIP tree-code against the CPU oracle (called through the C ABI).

Tolerances: FP64-expansion runs rel-L2 <= 1e-6 against the FP64 direct sum,
mixed runs (FP32 + Kahan near field and local evaluation) rel-L2 <= 1e-4; the
GPU all-pairs direct sum itself is held to 1e-12 (FP64) and 1e-6 (mixed).
Tree indexing is compared bit for bit with the reference quadtree.
"""

import math

import numpy as np
import pytest

from oracle import direct, fmm_ref, tree_ref
from workloads import generators as G

from gpu_common import rel_l2, rel_max, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_04398_amd as pp
    s = pp.Solver(0)
    yield s
    s.close()


def _case_random(seed, n=40, nt=500, zero_frac=0.3, h=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.standard_normal((n, n))
    f[rng.uniform(size=f.shape) < zero_frac] = 0.0
    h = h or 1.0 / n
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    tx = np.concatenate([x.ravel()[::3], 0.3 * n * h + 0.02 * n * h * rng.standard_normal(nt // 4),
                         rng.uniform(0, n * h, nt)])
    ty = np.concatenate([y.ravel()[::3], 0.6 * n * h + 0.02 * n * h * rng.standard_normal(nt // 4),
                         rng.uniform(0, n * h, nt)])
    tx = np.clip(tx, 0, n * h * (1 - 1e-12))
    ty = np.clip(ty, 0, n * h * (1 - 1e-12))
    return f, h, tx, ty


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_direct_gaussian64(solver, precision, tol):
    w = G.workload("gaussian64")
    g = w["grid"]
    ref = direct.direct_grid(w["f"], g.h, w["tx"], w["ty"])
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    P = to_host(solver.direct_grid(f, g.h, tx, ty, precision=precision))
    assert rel_l2(P, ref) < tol, rel_l2(P, ref)


@pytest.mark.parametrize("mode", ["skip", "cellavg"])
def test_direct_random_offgrid(solver, mode):
    f, h, tx, ty = _case_random(1)
    ref = direct.direct_grid(f, h, tx, ty, self_mode=1 if mode == "cellavg" else 0)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        P = solver.direct_grid(f, h, tx, ty, precision=prec, self_mode=mode, leaf_max=16)
        assert rel_l2(P, ref) < tol, (prec, rel_l2(P, ref))


def test_tree_bit_exact_gaussian64(solver):
    w = G.workload("gaussian64")
    g = w["grid"]
    solver.solve_grid(w["f"], g.h, w["tx"], w["ty"], p=8, theta=0.5, precision="fp64")
    info = tree_ref.grid_tree(w["f"], w["tx"], w["ty"], g.h, leaf_max=64)
    _compare_tree(solver, info, 0.5, 64)


def _compare_tree(solver, info, theta, nx):
    t = info["tree"]
    np.testing.assert_array_equal(solver.debug_array("SRC_KEY").astype(np.uint64), info["src_keys"])
    ij = solver.debug_array("SRC_INDEX").astype(np.int64)
    # packed (i | j << 16) versus the reference's flat j * nx + i
    assert np.array_equal((ij >> 16) * nx + (ij & 0xFFFF), info["src_flat"])
    np.testing.assert_array_equal(solver.debug_array("TGT_KEY").astype(np.uint64), info["tgt_keys"])
    np.testing.assert_array_equal(solver.debug_array("TGT_PERM"), info["tgt_perm"])
    for name, ref in (("CELL_LEVEL", t.level), ("CELL_IX", t.ix), ("CELL_IY", t.iy), ("CELL_SB", t.sb),
                      ("CELL_SE", t.se), ("CELL_TB", t.tb), ("CELL_TE", t.te), ("CELL_CHILD", t.child_begin),
                      ("CELL_NCHILD", t.nchild), ("CELL_PARENT", t.parent)):
        np.testing.assert_array_equal(solver.debug_array(name), ref, err_msg=name)
    m2l, p2p = tree_ref.interaction_lists(t, theta)
    for kind, ref_pairs in (("M2L", m2l), ("P2P", p2p)):
        off = solver.debug_array(kind + "_OFF")
        cnt = solver.debug_array(kind + "_CNT")
        src = solver.debug_array(kind + "_SRC")
        got = sorted((a, int(b)) for a in range(t.ncells) for b in src[off[a]:off[a] + cnt[a]])
        assert got == sorted(ref_pairs), kind


@pytest.mark.parametrize("seed,leaf_max,theta", [(1, 8, 0.5), (2, 16, 0.4), (3, 4, 0.6)])
def test_tree_bit_exact_adaptive(solver, seed, leaf_max, theta):
    f, h, tx, ty = _case_random(seed, n=48 if seed != 3 else 37)
    solver.solve_grid(f, h, tx, ty, p=6, theta=theta, leaf_max=leaf_max, precision="fp64")
    info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=leaf_max)
    _compare_tree(solver, info, theta, f.shape[1])


def test_tree_bit_exact_clustered_targets(solver):
    """Target starts of the dense prefix table when one workgroup's prefixes hold more targets than it
    stages in LDS (3,000 targets inside a 3 x 3-cell square, searched in global memory within the
    bracketed range) beside prefixes with few targets (1,000 spread ones, staged): the tree, the target
    order and the lists equal the oracle's."""
    n = 128
    h = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(77))
    f = rng.standard_normal((n, n))
    tx = np.concatenate([rng.uniform(0.40, 0.42, 3000), rng.uniform(0.0, 1.0, 1000)])
    ty = np.concatenate([rng.uniform(0.60, 0.62, 3000), rng.uniform(0.0, 1.0, 1000)])
    solver.solve_grid(f, h, tx, ty, p=6, theta=0.5, leaf_max=64, precision="fp64")
    info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=64)
    _compare_tree(solver, info, 0.5, n)


def test_target_sort_multi_tile(solver):
    """The target sort over many tiles with a ragged tail, a third of the targets repeated (equal keys,
    whose input order the stable sort keeps) and the rest spread: keys and permutation equal the
    oracle's stable sort."""
    n = 128
    h = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(41))
    f = rng.standard_normal((n, n))
    m = 3 * 4096 + 1234
    rep = rng.uniform(0.0, 1.0, (40, 2))[rng.integers(0, 40, m // 3)]
    tx = np.concatenate([rep[:, 0], rng.uniform(0.0, 1.0, m - m // 3)])
    ty = np.concatenate([rep[:, 1], rng.uniform(0.0, 1.0, m - m // 3)])
    solver.solve_grid(f, h, tx, ty, p=6, theta=0.5, leaf_max=64, precision="mixed")
    keys, perm = tree_ref.target_keys_sorted(tx, ty, 0.0, 0.0, h, tree_ref.root_exponent(n, n))
    np.testing.assert_array_equal(solver.debug_array("TGT_KEY").astype(np.uint64), keys)
    np.testing.assert_array_equal(solver.debug_array("TGT_PERM"), perm)


@pytest.mark.parametrize("ny,nx,m", [(2100, 2100, 32768), (3, 9000, 20000), (5, 5, 2), (128, 128, 70001)])
def test_target_sort_widths(ny, nx, m):
    """The target sort at several key widths: three passes of 8 bits at a 4096 root (32 tiles, offsets
    summed inside the scatter), four of 7 bits at 16384, one of 6 bits at 8, two of 7 bits over 69 tiles
    (offsets from a separate scan).  Keys and permutation equal the oracle's stable sort; a third of the
    targets share one of 40 positions (equal keys)."""
    import paper_1610_04398_amd as pp
    s = pp.Solver(0)
    try:
        rng = np.random.Generator(np.random.PCG64(nx + m))
        f = rng.standard_normal((ny, nx))
        h = 1.0 / max(nx, ny)
        rep = rng.uniform(0.0, 1.0, (40, 2))[rng.integers(0, 40, m // 3)]
        tx = np.concatenate([rep[:, 0], rng.uniform(0.0, 1.0, m - m // 3)]) * nx * h
        ty = np.concatenate([rep[:, 1], rng.uniform(0.0, 1.0, m - m // 3)]) * ny * h
        s.solve_grid(f, h, tx, ty, p=4, theta=0.5, leaf_max=64, precision="mixed")
        keys, perm = tree_ref.target_keys_sorted(tx, ty, 0.0, 0.0, h, tree_ref.root_exponent(nx, ny))
        np.testing.assert_array_equal(s.debug_array("TGT_KEY").astype(np.uint64), keys)
        np.testing.assert_array_equal(s.debug_array("TGT_PERM"), perm)
    finally:
        s.close()


@pytest.mark.parametrize("ny,nx,offset", [(40, 40, 0), (700, 1101, 0), (1030, 1030, 1), (2050, 2050, 0)])
def test_ingest_sources_bit_exact(solver, ny, nx, offset):
    """The grid ingest (nonzero counts per Morton tile of 64 x 32 nodes in groups of tiles, then emission of
    each tile at its offset) gives the oracle's sources bit for bit: one tile; an odd row length (node pairs
    loaded one by one) over 2,048 tiles in groups of two; f 8 bytes off 16-byte alignment; 8,192 tiles in
    groups of eight.  Zero patches leave whole tiles and groups empty."""
    import torch
    rng = np.random.Generator(np.random.PCG64(77 + nx + ny))
    f = rng.standard_normal((ny, nx))
    f[rng.uniform(size=f.shape) < 0.6] = 0.0
    f[: ny // 3, : nx // 2] = 0.0
    h = 1.0 / max(nx, ny)
    tx, ty = rng.uniform(0, nx * h, 300), rng.uniform(0, ny * h, 300)
    base = torch.zeros(nx * ny + offset, dtype=torch.float64, device="cuda")
    fd = base[offset:].view(ny, nx)
    fd.copy_(torch.from_numpy(f))
    assert (fd.data_ptr() % 16 == 0) == (offset == 0)
    solver.solve_grid(fd, h, *to_dev(tx, ty), p=6, theta=0.5, precision="mixed")
    ref_keys, ref_flat = tree_ref.source_keys_grid(f)
    np.testing.assert_array_equal(solver.debug_array("SRC_KEY").astype(np.uint64), ref_keys)
    ij = solver.debug_array("SRC_INDEX").astype(np.int64)
    assert np.array_equal((ij >> 16) * nx + (ij & 0xFFFF), ref_flat)
    assert solver.stats()["nsources"] == ref_keys.size


@pytest.mark.parametrize("dense_levels", ["0", "3"])
def test_tree_bit_exact_levelwise(monkeypatch, dense_levels):
    """The level-by-level construction (from the root, or below a shallow dense top) gives the same tree."""
    import paper_1610_04398_amd as pp
    monkeypatch.setenv("PP_DENSE_LEVELS", dense_levels)
    s = pp.Solver(0)
    try:
        f, h, tx, ty = _case_random(2, n=48)
        s.solve_grid(f, h, tx, ty, p=6, theta=0.4, leaf_max=16, precision="fp64")
        info = tree_ref.grid_tree(f, tx, ty, h, leaf_max=16)
        _compare_tree(s, info, 0.4, f.shape[1])
    finally:
        s.close()


def test_fmm_gaussian64_fp64(solver):
    w = G.workload("gaussian64")
    g = w["grid"]
    ref = direct.direct_grid(w["f"], g.h, w["tx"], w["ty"])
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    P = to_host(solver.solve_grid(f, g.h, tx, ty, p=8, theta=0.5, precision="fp64"))
    e = rel_l2(P, ref)
    assert e < 1e-6, e
    # same approximation as the FP64 reference tree-code, to rounding
    r = fmm_ref.fmm_grid(w["f"], w["tx"], w["ty"], g.h, 8, 0.5)
    assert rel_l2(P, r["P"]) < 1e-12


def test_fmm_per_pass_against_reference(solver):
    f, h, tx, ty = _case_random(4, n=32, nt=300)
    p = 10
    solver.solve_grid(f, h, tx, ty, p=p, theta=0.5, leaf_max=16, precision="fp64")
    r = fmm_ref.fmm_grid(f, tx, ty, h, p, 0.5, leaf_max=16)
    t = r["tree"]
    k = r["info"]["k"]
    mp = solver.debug_array("MULTIPOLE").reshape(t.ncells, p + 1, 2)
    loc = solver.debug_array("LOCAL").reshape(t.ncells, p + 1, 2)
    mpc = mp[..., 0] + 1j * mp[..., 1]
    locc = loc[..., 0] + 1j * loc[..., 1]
    for c in range(t.ncells):
        s = h * 2.0 ** (k - t.level[c])
        kk = np.arange(p + 1)
        if t.nsrc(c) > 0:
            # scaled a'_k = a_k / s^k with a_0 = S, a_k = -alpha_k
            ref_a = np.concatenate([[r["S"][c]], -r["alpha"][c][1:]]) / s**kk
            assert np.allclose(mpc[c], ref_a, rtol=1e-11, atol=1e-13 * abs(ref_a).max() + 1e-300), c
        if t.ntgt(c) > 0:
            ref_l = r["L"][c] * s**kk
            scale = np.abs(ref_l).max() + 1e-300
            assert np.max(np.abs(locc[c] - ref_l)) < 1e-10 * scale, c


def _case_leaf_widths(seed, n, sparse_zero):
    """Grid leaves of several widths: 8-node leaves (most of them, some nodes culled), wider leaves in a
    sparse quadrant (sparse_zero of its nodes zero), and 4-node leaves where a cluster of 150 targets splits
    an 8-node cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.standard_normal((n, n))
    f[rng.uniform(size=f.shape) < 0.3] = 0.0
    q = f[n // 2:, n // 2:]
    q[rng.uniform(size=q.shape) < sparse_zero] = 0.0
    h = 1.0 / n
    tx = np.concatenate([(8 + 8 * rng.uniform(size=150)) * h, rng.uniform(0, 1, 300)])
    ty = np.concatenate([(16 + 8 * rng.uniform(size=150)) * h, rng.uniform(0, 1, 300)])
    return f, h, np.clip(tx, 0, 1 - 1e-12), np.clip(ty, 0, 1 - 1e-12)


@pytest.mark.parametrize("lattice", ["1", "0"])
@pytest.mark.parametrize("n,p,sparse_zero", [(64, 12, 0.95), (64, 5, 0.95), (64, 17, 0.95), (128, 12, 0.85)])
def test_p2m_leaf_widths_against_reference(monkeypatch, lattice, n, p, sparse_zero):
    """P2M (Appendix A, eq. alphaK) of every source leaf, and M2M above it, against the reference
    expansions, with the matrix-core path forced for any number of leaves (grid leaves 8 nodes wide as a
    fixed contraction over their 64 node positions, leaves of other widths, 4, 16 and 32 nodes, in the same
    launch, several of them in one group of 16 leaves at 128^2) and with the lane groups for every leaf;
    p = 5, 12 and 17 (one, two and three 16-column tiles of coefficients)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_04398_amd as pp
    monkeypatch.setenv("PP_P2M_LATTICE", lattice)
    solver = pp.Solver(0)
    f, h, tx, ty = _case_leaf_widths(11 + n, n, sparse_zero)
    try:
        solver.solve_grid(f, h, tx, ty, p=p, theta=0.5, leaf_max=64, precision="fp64")
        _check_multipoles(solver, f, h, tx, ty, p)
    finally:
        solver.close()


def _check_multipoles(solver, f, h, tx, ty, p):
    """Every cell's scaled multipole coefficients against the reference FMM's, to 1e-11."""
    r = fmm_ref.fmm_grid(f, tx, ty, h, p, 0.5, leaf_max=64)
    t = r["tree"]
    k = r["info"]["k"]
    widths = {int(k - t.level[c]) for c in range(t.ncells) if t.leaf[c] and t.nsrc(c) > 0}
    assert {2, 3} <= widths and max(widths) >= 4, widths
    mp = solver.debug_array("MULTIPOLE").reshape(t.ncells, p + 1, 2)
    mpc = mp[..., 0] + 1j * mp[..., 1]
    kk = np.arange(p + 1)
    for c in range(t.ncells):
        if t.nsrc(c) == 0:
            continue
        s = h * 2.0 ** (k - t.level[c])
        ref_a = np.concatenate([[r["S"][c]], -r["alpha"][c][1:]]) / s**kk
        assert np.allclose(mpc[c], ref_a, rtol=1e-11, atol=1e-13 * abs(ref_a).max() + 1e-300), (c, t.level[c])


def test_mixed_l2p_is_compensated(solver):
    """The mixed path's FP32 L2P is a compensated Horner evaluation (u and the coefficients carried as FP32
    pairs).  Both precisions build the same FP64 local expansions, so the mixed far field must equal the
    FP64 path's to far better than FP32 rounding (< 1e-11), while a plain FP32 Horner evaluation of the
    reference FMM's locals misses the reference far field by ~4e-8; and both far fields match the reference
    FMM's (FP64 locals of a different summation order) to its own agreement, < 1e-8."""
    f, h, tx, ty = _case_random(4, n=32, nt=300)
    p = 10
    perm = None
    fars = {}
    for prec in ("fp64", "mixed"):
        solver.solve_grid(f, h, tx, ty, p=p, theta=0.5, leaf_max=16, precision=prec)
        perm = solver.debug_array("TGT_PERM")
        far = np.empty(tx.size)
        far[perm] = solver.debug_array("FAR") / (2 * math.pi)
        fars[prec] = far
    r = fmm_ref.fmm_grid(f, tx, ty, h, p, 0.5, leaf_max=16)
    t = r["tree"]
    k = r["info"]["k"]
    ref = r["far"]
    # plain FP32 Horner of the reference locals (scaled by the cell side) at the same points
    rperm = r["info"]["tgt_perm"]
    naive = np.empty(tx.size)
    for c in range(t.ncells):
        if not t.leaf[c] or t.ntgt(c) == 0:
            continue
        side = h * 2.0 ** (k - t.level[c])
        zc = complex((t.ix[c] + 0.5) * side, (t.iy[c] + 0.5) * side)
        for q in range(int(t.tb[c]), int(t.te[c])):
            u = (complex(tx[rperm[q]], ty[rperm[q]]) - zc) / side
            ux, uy = np.float32(u.real), np.float32(u.imag)
            ax, ay = np.float32(0), np.float32(0)
            for l in range(p, -1, -1):
                cl = r["L"][c][l] * side**l
                ax, ay = (np.float32(ax * ux - ay * uy + np.float32(cl.real)),
                          np.float32(ax * uy + ay * ux + np.float32(cl.imag)))
            naive[rperm[q]] = float(ax) / (2 * math.pi)
    e_comp = rel_l2(fars["mixed"], fars["fp64"])
    e_naive = rel_l2(naive, ref)
    e_ref = {prec: rel_l2(v, ref) for prec, v in fars.items()}
    print(f"far field: compensated FP32 vs FP64 {e_comp:.3e}, plain FP32 {e_naive:.3e}, vs reference {e_ref}")
    assert e_comp < 1e-11, e_comp
    assert e_comp * 1000 < e_naive, (e_comp, e_naive)
    assert max(e_ref.values()) < 1e-8, e_ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_fmm_random_cases(solver, precision, tol):
    for seed in (5, 6):
        for mode in ("skip", "cellavg"):
            f, h, tx, ty = _case_random(seed, n=64, nt=800)
            ref = direct.direct_grid(f, h, tx, ty, self_mode=1 if mode == "cellavg" else 0)
            P = solver.solve_grid(f, h, tx, ty, p=12, theta=0.5, leaf_max=32, precision=precision, self_mode=mode)
            assert rel_l2(P, ref) < tol, (seed, mode, rel_l2(P, ref))


def test_host_and_device_pointers_agree_and_deterministic(solver):
    f, h, tx, ty = _case_random(7, n=64)
    P1 = solver.solve_grid(f, h, tx, ty, precision="mixed")
    fd, txd, tyd = to_dev(f, tx, ty)
    P2 = to_host(solver.solve_grid(fd, h, txd, tyd, precision="mixed"))
    P3 = to_host(solver.solve_grid(fd, h, txd, tyd, precision="mixed"))
    assert np.array_equal(P1, P2) and np.array_equal(P2, P3)


# Observed on MI355X (all 264,192 targets of vortex512, against the oracle):
# mixed rel-L2 ~6e-8, rel-max ~1.5e-7; FP64 rel-L2 ~1e-10.  The bounds below
# sit about ten times above what the kernels reach, and far below the
# tolerances of the accuracy contract (rel-L2 1e-4 mixed, 1e-6 FP64), so a
# handful of wrong targets or a lost compensation fails them.
C2_BOUNDS = {"fp64": {"rel_l2": 1e-6, "rel_l2_tight": 2e-9, "rel_max": 1e-8},
             "mixed": {"rel_l2": 1e-4, "rel_l2_tight": 6e-7, "rel_max": 2e-6}}


def _group_errors(P, ref, n_grid):
    out = {}
    for name, sl in (("grid", slice(0, n_grid)), ("surface", slice(n_grid, None))):
        out[name] = {"rel_l2": rel_l2(P[sl], ref[sl]), "rel_max": rel_max(P[sl], ref[sl])}
    return out


def test_vortex512_full(solver):
    """The 512^2 vortex workload at full size against the oracle at every one of its 264,192 targets
    (262,144 grid nodes, 2,048 ellipse points), FP64 and mixed: rel-L2 separately over grid and surface
    targets, and the largest error of any single target relative to max |P|."""
    from oracle_cache import full_direct
    w = G.workload("vortex512")
    g = w["grid"]
    ref = full_direct("vortex512")
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    for prec in ("fp64", "mixed"):
        P = to_host(solver.solve_grid(f, g.h, tx, ty, p=12, theta=0.5, precision=prec))
        errs = _group_errors(P, ref, w["n_grid_targets"])
        print(f"vortex512 {prec}: {errs}")
        b = C2_BOUNDS[prec]
        for grp, e in errs.items():
            assert e["rel_l2"] < b["rel_l2"] and e["rel_l2"] < b["rel_l2_tight"], (prec, grp, e)
            assert e["rel_max"] < b["rel_max"], (prec, grp, e)


def test_vortex512_tree_bit_exact(solver):
    """Morton keys, the target permutation, every cell array and both interaction lists of the full
    vortex512 tree (5,733 cells) equal the reference quadtree's bit for bit."""
    w = G.workload("vortex512")
    g = w["grid"]
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    solver.solve_grid(f, g.h, tx, ty, p=12, theta=0.5, precision="mixed")
    info = tree_ref.grid_tree(w["f"], w["tx"], w["ty"], g.h, leaf_max=64)
    _compare_tree(solver, info, 0.5, g.nx)


def test_vortex512_kahan_near_field(solver):
    """Compensated FP32 near field (pin 11 of the accuracy contract): on the vortex512 lists, the
    library's mixed-precision near sums of 40 sampled target leaves (2,400+ targets, ~1,500 sources each)
    lie within 1e-6 (rel-L2) of the FP64 near sums over the same source sets, and are several times
    closer to them than a plain FP32 running sum of the same FP32 terms in the same part split."""
    from near_emulation import near_lists, near_sums
    w = G.workload("vortex512")
    g = w["grid"]
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    solver.solve_grid(f, g.h, tx, ty, p=12, theta=0.5, precision="mixed")
    near = solver.debug_array("NEAR")
    m = w["tx"].size
    parts = near.size // m
    gpu = near.reshape(parts, m).sum(axis=0)
    info = tree_ref.grid_tree(w["f"], w["tx"], w["ty"], g.h, leaf_max=64)
    lists = near_lists(info["tree"], 0.5)
    rng = np.random.Generator(np.random.PCG64(5))
    leaves = sorted(lists)
    pick = [leaves[i] for i in sorted(rng.choice(len(leaves), 40, replace=False))]
    ref, naive, idx = near_sums(w["f"], g.h, w["tx"], w["ty"], info, lists, pick, nparts=parts)
    e_gpu = rel_l2(gpu[idx], ref)
    e_naive = rel_l2(naive, ref)
    print(f"near field: compensated {e_gpu:.3e}, plain FP32 {e_naive:.3e} ({idx.size} targets)")
    assert e_gpu < 1e-6, e_gpu
    assert e_gpu * 5 < e_naive, (e_gpu, e_naive)


def test_kahan_near_field_sparse_target_leaves(solver):
    """The same pin for leaves that hold at most 16 targets (surface points over a grid source), where one
    lane per (target, source slot) sums strided sources: within 1e-6 of the FP64 near sums of the reference
    lists, and several times closer to them than a plain FP32 running sum."""
    from near_emulation import near_lists, near_sums
    n = 512
    g = G.GridSpec(n, n, 1.0 / n)
    f = G.vortex_source(g, 2)
    ex, ey = G.ellipse_targets(2048)
    sx, sy, lx, ly = G.fish_surface_targets(1024, g.h)
    tx, ty = np.concatenate([ex, sx, lx]), np.concatenate([ey, sy, ly])
    fd, txd, tyd = to_dev(f, tx, ty)
    solver.solve_grid(fd, g.h, txd, tyd, p=12, theta=0.5, precision="mixed")
    near = solver.debug_array("NEAR")
    parts = near.size // tx.size
    gpu = near.reshape(parts, tx.size).sum(axis=0)
    info = tree_ref.grid_tree(f, tx, ty, g.h, leaf_max=64)
    t = info["tree"]
    lists = near_lists(t, 0.5)
    sparse = [a for a in sorted(lists) if 0 < t.te[a] - t.tb[a] <= 16]
    assert len(sparse) >= 60
    rng = np.random.Generator(np.random.PCG64(6))
    pick = [sparse[i] for i in sorted(rng.choice(len(sparse), 60, replace=False))]
    ref, naive, idx = near_sums(f, g.h, tx, ty, info, lists, pick, nparts=parts)
    e_gpu = rel_l2(gpu[idx], ref)
    e_naive = rel_l2(naive, ref)
    print(f"sparse leaves near field: compensated {e_gpu:.3e}, plain FP32 {e_naive:.3e} ({idx.size} targets)")
    assert e_gpu < 1e-6, e_gpu
    assert e_gpu * 3 < e_naive, (e_gpu, e_naive)


def test_error_paths_leave_output_untouched(solver):
    import paper_1610_04398_amd as pp
    f, h, tx, ty = _case_random(8, n=16, nt=20)
    out = np.full(tx.size, 7.0)
    with pytest.raises(pp.PPError) as e:
        solver.solve_grid(f, h, np.concatenate([tx[:-1], [2.0]]), ty, out=out)
    assert e.value.status == -2 and np.all(out == 7.0)
    with pytest.raises(pp.PPError) as e:  # a non-finite target coordinate
        solver.solve_grid(f, h, tx, np.concatenate([ty[:-1], [np.nan]]), out=out)
    assert e.value.status == -1 and np.all(out == 7.0)
    bad = f.copy()
    bad[3, 4] = np.nan
    with pytest.raises(pp.PPError) as e:
        solver.solve_grid(bad, h, tx, ty, out=out)
    assert e.value.status == -1 and np.all(out == 7.0)
    with pytest.raises(pp.PPError) as e:
        solver.solve_grid(f, h, tx, ty, p=0, out=out)
    assert e.value.status == -1
    with pytest.raises(pp.PPError) as e:
        solver.solve_grid(f, h, tx, ty, theta=1.0, out=out)
    assert e.value.status == -1
    with pytest.raises(pp.PPError) as e:
        solver.solve_grid(f, -h, tx, ty, out=out)
    assert e.value.status == -1
    assert np.all(out == 7.0)


def test_budget_exceeded_before_any_work():
    """A context whose device-memory budget is too small for a solve returns PP_ERR_NOMEM before it
    allocates or launches anything: the output is untouched, the context holds no new memory, and it
    still solves a problem that fits the budget."""
    import paper_1610_04398_amd as pp
    budget = 256 << 10  # a 16^2 solve fits, a 128^2 one (about 3 MB) does not
    s = pp.Solver(0, hbm_budget_bytes=budget)
    try:
        f, h, tx, ty = _case_random(8, n=128, nt=2000)
        out = np.full(tx.size, 7.0)
        with pytest.raises(pp.PPError) as e:
            s.solve_grid(f, h, tx, ty, out=out)
        assert e.value.status == -3 and np.all(out == 7.0)
        assert "budget" in str(e.value)
        small, hs, sx, sy = _case_random(9, n=16, nt=50)
        got = s.solve_grid(small, hs, sx, sy, precision="fp64")
        assert rel_l2(got, direct.direct_grid(small, hs, sx, sy)) < 1e-6
    finally:
        s.close()


def test_degenerate_inputs(solver):
    # all-zero sources: P == 0
    f = np.zeros((8, 8))
    tx = np.array([0.1, 0.5, 0.93])
    ty = np.array([0.2, 0.5, 0.01])
    assert np.all(solver.solve_grid(f, 1 / 8, tx, ty) == 0.0)
    # single node, single target on it (skip -> 0, cellavg -> w (ln h - kappa) / 2pi)
    f1 = np.array([[2.0]])
    assert solver.solve_grid(f1, 0.5, [0.25], [0.25], precision="fp64")[0] == 0.0
    v = solver.solve_grid(f1, 0.5, [0.25], [0.25], precision="fp64", self_mode="cellavg")[0]
    kappa = 1.5 - math.pi / 4 + 0.5 * math.log(2)
    assert abs(v - 0.5 * (math.log(0.5) - kappa) / (2 * math.pi)) < 1e-15
    # no targets
    assert solver.solve_grid(f1, 0.5, np.zeros(0), np.zeros(0)).size == 0
    # non-square, non-power-of-two grid with a ragged tail
    rng = np.random.Generator(np.random.PCG64(9))
    f2 = rng.standard_normal((37, 101))
    h = 0.01
    tx = rng.uniform(0, 1.27, 400)
    ty = rng.uniform(0, 1.27, 400)
    ref = direct.direct_grid(f2, h, tx, ty)
    for prec, tol in (("fp64", 1e-6), ("mixed", 1e-4)):
        P = solver.solve_grid(f2, h, tx, ty, precision=prec, leaf_max=16)
        assert rel_l2(P, ref) < tol
    # targets within 2^-20 h of a node but not on it, and exactly on it
    g = G.GridSpec(16, 16, 1 / 16)
    f3 = rng.standard_normal((16, 16))
    x, y = G.grid_nodes(g)
    tx = np.array([x[3, 5], x[3, 5] + 1e-9, x[7, 2] - 3e-12, 0.5])
    ty = np.array([y[3, 5], y[3, 5], y[7, 2] + 1e-10, 0.5])
    ref = direct.direct_grid(f3, 1 / 16, tx, ty)
    # all-pairs GPU sum: the snapped node's exact FP64 term is restored
    P = solver.direct_grid(f3, 1 / 16, tx, ty, precision="fp64", leaf_max=8)
    assert rel_max(P, ref) < 1e-12
    # mixed: the near-coincident target is snapped (moved by < 2^-20 h)
    P = solver.direct_grid(f3, 1 / 16, tx, ty, precision="mixed", leaf_max=8)
    assert rel_max(P, ref) < 2e-6
    # tree-code: truncation error only
    P = solver.solve_grid(f3, 1 / 16, tx, ty, precision="fp64", leaf_max=8)
    assert rel_max(P, ref) < 1e-7
    P = solver.solve_grid(f3, 1 / 16, tx, ty, precision="mixed", leaf_max=8)
    assert rel_max(P, ref) < 1e-5


def _sampled_check(solver, name, n_samples=600, seed=21):
    """rel-L2 and largest single-target error (relative to max |P| of the sample) of FP64 and mixed solves
    on seeded sampled targets, against the oracle evaluated at those targets one by one."""
    w = G.workload(name)
    g = w["grid"]
    rng = np.random.Generator(np.random.PCG64(seed))
    sel = rng.choice(w["tx"].size, n_samples, replace=False)
    ref = direct.direct_grid(w["f"], g.h, w["tx"][sel], w["ty"][sel])
    f, tx, ty = to_dev(w["f"], w["tx"], w["ty"])
    errs = {}
    for prec in ("fp64", "mixed"):
        P = to_host(solver.solve_grid(f, g.h, tx, ty, p=w["p"], theta=w["theta"], precision=prec))
        errs[prec] = {"rel_l2": rel_l2(P[sel], ref), "rel_max": rel_max(P[sel], ref)}
    print(f"{name}: {errs}")
    return w, errs


# Observed on MI355X at the sampled targets (rel-L2 / largest error relative to max |P|):
# band2048 (p = 16, theta = 0.4) FP64 2.6e-14 / 1.2e-13, mixed 3.6e-8 / 7.3e-8;
# envelope4096 (p = 12, theta = 0.5) FP64 1.9e-11 / 8.5e-11, mixed 3.3e-8 / 5.0e-8.
# The bounds sit about ten times above.
SAMPLED_BOUNDS = {"band2048": {"fp64": (3e-13, 1.5e-12), "mixed": (4e-7, 8e-7)},
                  "envelope4096": {"fp64": (2e-10, 1e-9), "mixed": (4e-7, 6e-7)}}


def _check_bounds(name, errs):
    for prec, (b_l2, b_max) in SAMPLED_BOUNDS[name].items():
        tol = 1e-6 if prec == "fp64" else 1e-4
        e = errs[prec]
        assert e["rel_l2"] < tol and e["rel_l2"] < b_l2 and e["rel_max"] < b_max, (name, prec, e)


def test_band2048_sampled(solver):
    """2048^2 band-masked vortex source, 16,384 surface/lifted targets, p=16, theta=0.4."""
    w, errs = _sampled_check(solver, "band2048")
    _check_bounds("band2048", errs)
    # the tree of this adaptive case against the reference: arrays in full, lists on sampled cells
    info = tree_ref.grid_tree(w["f"], w["tx"], w["ty"], w["grid"].h, leaf_max=64)
    t = info["tree"]
    np.testing.assert_array_equal(solver.debug_array("TGT_PERM"), info["tgt_perm"])
    for name, ref in (("CELL_LEVEL", t.level), ("CELL_IX", t.ix), ("CELL_IY", t.iy), ("CELL_SB", t.sb),
                      ("CELL_SE", t.se), ("CELL_TB", t.tb), ("CELL_TE", t.te), ("CELL_CHILD", t.child_begin)):
        np.testing.assert_array_equal(solver.debug_array(name), ref, err_msg=name)
    rng = np.random.Generator(np.random.PCG64(3))
    tc = np.flatnonzero(t.te > t.tb)
    off = {k: solver.debug_array(k) for k in ("M2L_OFF", "M2L_CNT", "M2L_SRC", "P2P_OFF", "P2P_CNT", "P2P_SRC")}
    for a in rng.choice(tc, min(150, tc.size), replace=False):
        lm, lp = tree_ref.lists_for_cell(t, int(a), w["theta"])
        got_m = sorted(off["M2L_SRC"][off["M2L_OFF"][a]:off["M2L_OFF"][a] + off["M2L_CNT"][a]].tolist())
        got_p = sorted(off["P2P_SRC"][off["P2P_OFF"][a]:off["P2P_OFF"][a] + off["P2P_CNT"][a]].tolist())
        assert got_m == lm and got_p == lp, a


def test_envelope4096_sampled(solver):
    """4096^2 two-band envelope source (6.16M nonzero), 32,768 surface/lifted targets, p=12, theta=0.5.
    Accuracy on sampled targets; the tree (depth 12, ~130k cells) against the reference quadtree: keys,
    permutation and every cell array in full, the interaction lists on sampled target cells."""
    w, errs = _sampled_check(solver, "envelope4096", n_samples=400)
    _check_bounds("envelope4096", errs)
    st = solver.stats()
    assert st["nsources"] == int(np.count_nonzero(w["f"]))
    info = tree_ref.grid_tree(w["f"], w["tx"], w["ty"], w["grid"].h, leaf_max=64)
    t = info["tree"]
    np.testing.assert_array_equal(solver.debug_array("SRC_KEY").astype(np.uint64), info["src_keys"])
    ij = solver.debug_array("SRC_INDEX").astype(np.int64)
    assert np.array_equal((ij >> 16) * w["grid"].nx + (ij & 0xFFFF), info["src_flat"])
    np.testing.assert_array_equal(solver.debug_array("TGT_KEY").astype(np.uint64), info["tgt_keys"])
    np.testing.assert_array_equal(solver.debug_array("TGT_PERM"), info["tgt_perm"])
    for name, ref in (("CELL_LEVEL", t.level), ("CELL_IX", t.ix), ("CELL_IY", t.iy), ("CELL_SB", t.sb),
                      ("CELL_SE", t.se), ("CELL_TB", t.tb), ("CELL_TE", t.te), ("CELL_CHILD", t.child_begin),
                      ("CELL_NCHILD", t.nchild), ("CELL_PARENT", t.parent)):
        np.testing.assert_array_equal(solver.debug_array(name), ref, err_msg=name)
    rng = np.random.Generator(np.random.PCG64(7))
    tc = np.flatnonzero(t.te > t.tb)
    off = {k: solver.debug_array(k) for k in ("M2L_OFF", "M2L_CNT", "M2L_SRC", "P2P_OFF", "P2P_CNT", "P2P_SRC")}
    for a in rng.choice(tc, min(200, tc.size), replace=False):
        lm, lp = tree_ref.lists_for_cell(t, int(a), w["theta"])
        got_m = sorted(off["M2L_SRC"][off["M2L_OFF"][a]:off["M2L_OFF"][a] + off["M2L_CNT"][a]].tolist())
        got_p = sorted(off["P2P_SRC"][off["P2P_OFF"][a]:off["P2P_OFF"][a] + off["P2P_CNT"][a]].tolist())
        assert got_m == lm and got_p == lp, a


def test_list_modes_agree_bitwise(solver, monkeypatch):
    """One-pass lists (fixed capacity), their overflow fallback and two-pass lists give identical bits."""
    import paper_1610_04398_amd as pp
    f, h, tx, ty = _case_random(11, n=64, nt=900)
    ref = solver.solve_grid(f, h, tx, ty, p=10, theta=0.5, leaf_max=16, precision="mixed")
    for env in ({"PP_EXACT_LISTS": "1"}, {"PP_LIST_CAPS": "3,2"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        s2 = pp.Solver(0)
        got = s2.solve_grid(f, h, tx, ty, p=10, theta=0.5, leaf_max=16, precision="mixed")
        again = s2.solve_grid(f, h, tx, ty, p=10, theta=0.5, leaf_max=16, precision="mixed")
        s2.close()
        for k in env:
            monkeypatch.delenv(k)
        assert np.array_equal(got, ref) and np.array_equal(again, ref), env


@pytest.mark.parametrize("exact_lists", ["0", "1"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 1e-5)])
def test_large_target_leaf_beside_fine_sources(monkeypatch, precision, tol, exact_lists):
    """Targets only in the empty half of a half-filled source grid (leaf_max 1) sit in a target leaf a
    quarter of the domain wide beside source leaves of the finest level.  Almost no source cell is
    accepted for it, so its near list holds nearly every source leaf, and the traversal below it needs a
    longer stack than the smallest frontier tier holds: the first solve repeats at the next tier, a second
    call starts there, and both match the oracle's FMM and each other bit for bit.  Run with the one-pass
    lists and with the two-pass lists (count, then emit), whose count pass meets the overflow."""
    import paper_1610_04398_amd as pp
    monkeypatch.setenv("PP_EXACT_LISTS", exact_lists)
    n = 128
    rng = np.random.Generator(np.random.PCG64(31))
    f = rng.standard_normal((n, n))
    f[:, n // 2:] = 0.0
    h = 1.0 / n
    tx = np.array([0.75, 0.8, 0.9])
    ty = np.array([0.5, 0.6, 0.7])
    ref = fmm_ref.fmm_grid(f, tx, ty, h, 10, 0.5, leaf_max=1)["P"]
    exact = direct.direct_grid(f, h, tx, ty)
    s = pp.Solver(0)
    try:
        kw = dict(p=10, theta=0.5, leaf_max=1, precision=precision)
        first = s.solve_grid(f, h, tx, ty, **kw)
        second = s.solve_grid(f, h, tx, ty, **kw)
    finally:
        s.close()
    assert np.array_equal(first, second)
    assert rel_max(first, ref) < tol, rel_max(first, ref)
    assert rel_max(first, exact) < 1e-6


@pytest.mark.parametrize("near_stream,direct_issue,lists", [("1", "1", "onepass"), ("1", "0", "onepass"),
                                                             ("0", "1", "onepass"), ("1", "1", "exact"),
                                                             ("1", "1", "overflow")])
def test_graph_replay_matches_eager(monkeypatch, near_stream, direct_issue, lists):
    """Repeated solves on device inputs replay captured graphs (same shape and pointers; the second segment
    also needs the same tree).  Every call, with eager device work and synchronisations in between and with
    the source changed in place (same and different zero pattern), equals a context without replay and with
    every phase on one stream, bit for bit; with the near field on its own stream (the second segment issued
    directly, or forked and joined inside its graph) and without.  The two-pass lists (forced, or the retry
    after a one-pass list outgrew a tiny capacity) are emitted on the caller's stream before the near field
    starts on the side stream, which must wait for them."""
    import torch
    import paper_1610_04398_amd as pp
    n = 128
    g = G.GridSpec(n, n, 1.0 / n)
    base = G.vortex_source(g, 21, 16)
    rng = np.random.Generator(np.random.PCG64(22))
    tx = rng.uniform(0, 1, 3000)
    ty = rng.uniform(0, 1, 3000)
    fd, txd, tyd = to_dev(base, tx, ty)
    out = torch.empty(tx.size, dtype=torch.float64, device="cuda")
    monkeypatch.setenv("PP_GRAPHS", "0")
    monkeypatch.setenv("PP_NEAR_STREAM", "0")
    eager = pp.Solver(0)
    monkeypatch.delenv("PP_GRAPHS")
    monkeypatch.setenv("PP_NEAR_STREAM", near_stream)
    monkeypatch.setenv("PP_DIRECT_ISSUE", direct_issue)
    if lists == "exact":
        monkeypatch.setenv("PP_EXACT_LISTS", "1")
    elif lists == "overflow":
        monkeypatch.setenv("PP_LIST_CAPS", "3,2")
    fast = pp.Solver(0)
    for k in ("PP_NEAR_STREAM", "PP_DIRECT_ISSUE", "PP_EXACT_LISTS", "PP_LIST_CAPS"):
        monkeypatch.delenv(k, raising=False)
    kw = dict(p=12, theta=0.5, leaf_max=32, precision="mixed")
    try:
        for it in range(10):
            if it == 3:
                fd.mul_(1.5)                      # same zero pattern: same tree
            if it == 5:
                fd[: n // 2].zero_()              # different sources: a different tree
            if it == 7:
                fast.set_profiling(2)             # near field timed between replayed segments
            scratch = torch.randn(1 << 16, device="cuda").sum()  # eager device work between replays
            torch.cuda.synchronize()
            got = to_host(fast.solve_grid(fd, g.h, txd, tyd, out=out, **kw)).copy()
            ref = to_host(eager.solve_grid(fd, g.h, txd, tyd, **kw))
            assert np.array_equal(got, ref), it
            assert fast.stats()["n_p2p_pairs"] == eager.stats()["n_p2p_pairs"]
            if it >= 7:
                assert fast.stats()["ms_phase"]["p2p"] > 0.0
            del scratch
    finally:
        fast.close()
        eager.close()


@pytest.mark.parametrize("method,precision", [("fmm", "mixed"), ("fmm", "fp64"), ("treecode", "mixed")])
def test_lazy_packing_matches_full(monkeypatch, method, precision):
    """Few targets beside many source leaves (a 512^2 vortex source, 600 targets on an ellipse): the near
    field's source leaves are packed only when some list holds them (claimed once, queued, packed one wave
    each).  The cold and the resident solve equal, bit for bit, those of a context that packs every leaf."""
    import paper_1610_04398_amd as pp
    n = 512
    g = G.GridSpec(n, n, 1.0 / n)
    f = G.vortex_source(g, 31, 24)
    tx, ty = G.ellipse_targets(600)
    kw = dict(p=12, theta=0.5, leaf_max=64, precision=precision, method=method)
    monkeypatch.setenv("PP_LAZY_PACK", "0")
    full = pp.Solver(0)
    monkeypatch.delenv("PP_LAZY_PACK")
    lazy = pp.Solver(0)
    try:
        fd, txd, tyd = to_dev(f, tx, ty)
        a = to_host(lazy.solve_grid(fd, g.h, txd, tyd, **kw))
        b = to_host(full.solve_grid(fd, g.h, txd, tyd, **kw))
        assert np.array_equal(a, b)
        st = lazy.stats()
        assert 4 * st["ntgt_leaves"] < st["nsrc_leaves"]  # the lazy schedule is the one taken
        f2d = to_dev(1.3 * f)[0]
        a = to_host(lazy.solve_grid_resident(f2d, txd, tyd))
        b = to_host(full.solve_grid_resident(f2d, txd, tyd))
        assert np.array_equal(a, b)
        ref = direct.direct_grid(1.3 * f, g.h, tx, ty)
        assert rel_l2(a, ref) < (1e-6 if precision == "mixed" else 1e-8)
    finally:
        lazy.close()
        full.close()
