"""Pins of the FP64 expansion operators and the slow reference tree-code.

Operators follow Appendix A (eq. alphaK, eq. pressTruncated, eq. expandedShift /
eq. expandedBeta) and the local-expansion operators derived from eq.
logExpansion.  Pins: the multipole re-centring is exact (and the printed sign
of its S term is not), the local shift is exact, the truncation error obeys the
bound implied by the convergence condition of eq. logExpansion, and the whole
tree-code converges to the direct sum as p grows.
"""

import math

import numpy as np

from oracle import direct, fmm_ref
from workloads import generators as G


def _cluster(seed, n=50, centre=0.3 + 0.2j, rad=0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    z = centre + rad * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))
    w = rng.standard_normal(n)
    return z, w


def test_m2m_is_exact():
    """M2M of the children's P2M equals P2M about the parent for every k <= p (pin of eq. expandedBeta)."""
    p = 14
    zp = 0.5 + 0.5j
    S_tot = 0.0
    beta_tot = np.zeros(p + 1, complex)
    zs_all, ws_all = [], []
    for q, zc in enumerate((0.25 + 0.25j, 0.75 + 0.25j, 0.25 + 0.75j, 0.75 + 0.75j)):
        z, w = _cluster(q, centre=zc, rad=0.25)
        zs_all.append(z)
        ws_all.append(w)
        S, a = fmm_ref.p2m(z, w, zc, p)
        S2, b = fmm_ref.m2m(S, a, zc, zp)
        S_tot += S2
        beta_tot += b
    S_ref, a_ref = fmm_ref.p2m(np.concatenate(zs_all), np.concatenate(ws_all), zp, p)
    assert abs(S_tot - S_ref) < 1e-13 * abs(S_ref)
    assert np.max(np.abs(beta_tot - a_ref)) < 1e-13 * np.max(np.abs(a_ref))


def test_printed_m2m_sign_is_not_exact():
    """With the S term's sign as printed, the shifted coefficients miss P2M(parent) by O(1)."""
    p = 8
    z, w = _cluster(3, centre=0.25 + 0.25j, rad=0.2)
    w = np.abs(w) + 0.5  # nonzero total S
    S, a = fmm_ref.p2m(z, w, 0.25 + 0.25j, p)
    _, b = fmm_ref.m2m(S, a, 0.25 + 0.25j, 0.5 + 0.5j)
    z0 = -0.25 - 0.25j
    printed = b.copy()
    for k in range(1, p + 1):
        printed[k] = b[k] - 2.0 * S * z0**k / k
    _, ref = fmm_ref.p2m(z, w, 0.5 + 0.5j, p)
    assert np.max(np.abs(b - ref)) < 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(printed - ref)) > 1e-2 * np.max(np.abs(ref))


def test_l2l_is_exact():
    """Re-centring a local expansion reproduces the same polynomial everywhere."""
    rng = np.random.Generator(np.random.PCG64(1))
    L = rng.standard_normal(11) + 1j * rng.standard_normal(11)
    zc, zn = 0.3 - 0.1j, 0.35 - 0.05j
    L2 = fmm_ref.l2l(L, zc, zn)
    z = zn + 0.05 * (rng.uniform(-1, 1, 30) + 1j * rng.uniform(-1, 1, 30))
    a = fmm_ref.l2p(L, zc, z)
    b = fmm_ref.l2p(L2, zn, z)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_multipole_truncation_bound():
    """|Phi - Phi_p| <= A/(p+1) c^-p / (c-1), A = sum|w|, c = |z - zc| / max|z_i - zc| (from eq. logExpansion)."""
    for seed in range(6):
        z, w = _cluster(seed, n=40, centre=0.0, rad=0.1)
        r = np.max(np.abs(z))
        A = float(np.sum(np.abs(w)))
        rng = np.random.Generator(np.random.PCG64(100 + seed))
        zt = (rng.uniform(2.0, 8.0, 20) * r) * np.exp(1j * rng.uniform(0, 2 * math.pi, 20))
        exact = direct.direct_points(z.real, z.imag, w, zt.real, zt.imag)
        for p in (2, 5, 9, 14):
            S, a = fmm_ref.p2m(z, w, 0.0, p)
            approx = fmm_ref.m2p(S, a, 0.0, zt)
            c = np.abs(zt) / r
            bound = A / (p + 1) * c ** (-p) / (c - 1) / (2 * math.pi)
            assert np.all(np.abs(approx - exact) <= bound * (1 + 1e-9) + 1e-15)


def test_m2l_matches_multipole_evaluation():
    """The local expansion from M2L agrees with evaluating the multipole directly, error falling with p."""
    z, w = _cluster(9, n=30, centre=0.0, rad=0.05)
    zt_c = 0.4 + 0.1j
    rng = np.random.Generator(np.random.PCG64(2))
    zt = zt_c + 0.05 * (rng.uniform(-1, 1, 25) + 1j * rng.uniform(-1, 1, 25))
    exact = direct.direct_points(z.real, z.imag, w, zt.real, zt.imag)
    errs = []
    for p in (4, 8, 12, 16):
        S, a = fmm_ref.p2m(z, w, 0.0, p)
        L = fmm_ref.m2l(S, a, 0.0, zt_c, p)
        errs.append(np.max(np.abs(fmm_ref.l2p(L, zt_c, zt) - exact)))
    assert errs[-1] < 1e-12 * np.max(np.abs(exact))
    assert all(errs[i + 1] < errs[i] * 0.1 for i in range(len(errs) - 1))


def test_reference_fmm_vs_direct_gaussian64():
    """64^2 Gaussian, p = 8, theta = 0.5: within the FP64 tolerance 1e-6 of the direct sum, error falling with p."""
    w = G.workload("gaussian64")
    g = w["grid"]
    P = direct.direct_grid(w["f"], g.h, w["tx"], w["ty"])
    e = []
    for p in (4, 8):
        r = fmm_ref.fmm_grid(w["f"], w["tx"], w["ty"], g.h, p, 0.5)
        e.append(np.linalg.norm(r["P"] - P) / np.linalg.norm(P))
    assert e[1] < 1e-7
    assert e[1] < e[0] / 50


def test_reference_fmm_off_grid_targets_and_cellavg():
    rng = np.random.Generator(np.random.PCG64(8))
    n = 32
    h = 1.0 / n
    f = rng.standard_normal((n, n))
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    tx = np.concatenate([x.ravel()[::3], rng.uniform(0, 1, 200)])
    ty = np.concatenate([y.ravel()[::3], rng.uniform(0, 1, 200)])
    for mode in (0, 1):
        P = direct.direct_grid(f, h, tx, ty, self_mode=mode)
        r = fmm_ref.fmm_grid(f, tx, ty, h, 12, 0.5, leaf_max=16, self_mode=mode)
        assert np.linalg.norm(r["P"] - P) / np.linalg.norm(P) < 1e-9


def test_treecode_converges_to_direct():
    """The paper's tree-code (M2P at the targets, no locals) on random grid sources with off-grid and
    node targets: error falls geometrically with p and is within the FP64 tolerance at p = 12."""
    rng = np.random.Generator(np.random.PCG64(12))
    n = 32
    h = 1.0 / n
    f = rng.standard_normal((n, n))
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    tx = np.concatenate([x.ravel()[::5], rng.uniform(0, 1, 150)])
    ty = np.concatenate([y.ravel()[::5], rng.uniform(0, 1, 150)])
    P = direct.direct_grid(f, h, tx, ty)
    errs = []
    for p in (4, 8, 12):
        r = fmm_ref.treecode_grid(f, tx, ty, h, p, 0.5, leaf_max=16)
        errs.append(np.linalg.norm(r["P"] - P) / np.linalg.norm(P))
    assert errs[2] < 1e-6
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10


def test_treecode_far_part_obeys_the_m2p_bound():
    """For one target leaf, the M2P sum over its accepted cells differs from the direct sum over their
    sources by at most sum_B A_B / (p+1) c_B^-p / (c_B - 1), c_B = d / r_B (truncation of eq. pressTruncated)."""
    rng = np.random.Generator(np.random.PCG64(13))
    n = 32
    h = 1.0 / n
    f = rng.standard_normal((n, n))
    x, y = G.grid_nodes(G.GridSpec(n, n, h))
    tx, ty = x.ravel()[::7], y.ravel()[::7]
    p = 6
    r = fmm_ref.treecode_grid(f, tx, ty, h, p, 0.5, leaf_max=16)
    t, info = r["tree"], r["info"]
    k = info["k"]
    flat = info["src_flat"]
    sx = (flat % n + 0.5) * h
    sy = (flat // n + 0.5) * h
    w = f.ravel()[flat] * h * h
    perm = info["tgt_perm"]
    checked = 0
    for a, (m2p, _) in r["lists"].items():
        if not m2p:
            continue
        tl = perm[int(t.tb[a]):int(t.te[a])]
        for j in tl:
            zt = tx[j] + 1j * ty[j]
            approx = exact = bound = 0.0
            for b in m2p:
                side = h * 2.0 ** (k - int(t.level[b]))
                zc = complex((int(t.ix[b]) + 0.5) * side, (int(t.iy[b]) + 0.5) * side)
                approx += fmm_ref.m2p(r["S"][b], r["alpha"][b], zc, zt)
                sl = slice(int(t.sb[b]), int(t.se[b]))
                exact += np.sum(w[sl] * np.log(np.abs(zt - (sx[sl] + 1j * sy[sl])))) / (2 * math.pi)
                rad = side / math.sqrt(2)
                c = abs(zt - zc) / rad
                bound += np.sum(np.abs(w[sl])) / (p + 1) * c ** (-p) / (c - 1) / (2 * math.pi)
            assert abs(approx - exact) <= bound * (1 + 1e-9) + 1e-15
            checked += 1
    assert checked > 20
