"""Pins of the FP64 oracle against closed forms, brute force and invariants.

None of these checks re-runs the oracle's own formula: each compares it with a
special case that reduces to a textbook result (cubic d-spacings, sums of three
squares, rock-salt and fcc/bcc extinction rules, Lorentz-polarisation at
special angles), a brute-force high-precision evaluation, or an invariance the
physics guarantees (Friedel pairs, translations, unimodular basis changes,
supercells).
"""

import itertools
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2602_11709_amd import synth

LAM = synth.CU_KA


def r3(n):
    """Number of integer triples with h^2 + k^2 + l^2 = n (brute force)."""
    m = int(math.isqrt(n)) + 1
    return sum(1 for h in range(-m, m + 1) for k in range(-m, m + 1) for l in range(-m, m + 1)
               if h * h + k * k + l * l == n)


def cubic(a, frac, species, coeff, bfac=0.0, occ=None, tmin=0.0, tmax=90.0, lam=LAM):
    n = len(frac)
    return synth.CrystalBatch(
        name="t", lattice=np.array([[a, a, a, 90.0, 90.0, 90.0]]),
        atom_offset=np.array([0, n], np.int64), frac=np.asarray(frac, float).reshape(-1, 3),
        species=np.asarray(species, np.int32), occ=np.ones(n) if occ is None else np.asarray(occ, float),
        bfac=np.full(n, bfac) if np.isscalar(bfac) else np.asarray(bfac, float),
        sf_coeff=np.asarray(coeff, float), wavelength=lam, two_theta_min=np.array([tmin]),
        two_theta_max=np.array([tmax]))


# ---- scattering factor, LP, geometry ----------------------------------------

@pytest.mark.parametrize("i", range(4))
def test_fsc_single_gaussian_halves_at_ln2(i):
    # a_i exp(-ln2 * s^2) at s^2 = 1 is a_i / 2; other terms zero: catches a/b
    # index mix-ups and the sign of the exponent.
    coeff = np.zeros(9)
    coeff[i] = 3.0 + i
    coeff[4 + i] = math.log(2.0)
    assert oracle.fsc(coeff, 1.0) == pytest.approx((3.0 + i) / 2.0, rel=1e-15)
    assert oracle.fsc(coeff, 2.0) == pytest.approx((3.0 + i) / 4.0, rel=1e-15)


def test_fsc_limits():
    coeff = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 0.25])
    assert oracle.fsc(coeff, 0.0) == pytest.approx(10.25, rel=1e-15)  # sum a + c
    assert oracle.fsc(coeff, 1e4) == pytest.approx(0.25, rel=1e-15)   # -> c


@pytest.mark.parametrize("tt,val", [(90.0, 2.0 * math.sqrt(2.0)),
                                    (60.0, 1.25 / (0.25 * math.sqrt(3.0) / 2.0)),
                                    (120.0, 1.25 / (0.75 * 0.5)),
                                    (180.0 - 1e-12, None)])
def test_lp_special_angles(tt, val):
    # (1 + cos^2 2t)/(sin^2 t cos t) at 2t = 90: 1/(1/2 * 1/sqrt2) = 2 sqrt2, etc.
    if val is None:
        assert oracle.lp(tt) > 1e10  # cos(theta) -> 0 at back-scattering
    else:
        assert oracle.lp(tt) == pytest.approx(val, rel=1e-14)


def test_cubic_metric_and_bragg_positions():
    # Cubic: d = a / sqrt(h^2 + k^2 + l^2); the oracle goes through the general
    # triclinic metric inverse.
    a = 5.64
    g = oracle.cell([a, a, a, 90, 90, 90])
    assert g is not None
    _, gs, vol = g
    assert vol == pytest.approx(a ** 3, rel=1e-14)
    mp.mp.dps = 30
    for n in [1, 2, 3, 4, 8, 11, 12, 16, 19, 20, 24, 26]:
        h, k, l = next(t for t in itertools.product(range(6), repeat=3) if sum(x * x for x in t) == n)
        q = oracle.q_of(gs, h, k, l)
        assert q == pytest.approx(n / a ** 2, rel=1e-14)
        exact = 2 * mp.asin(mp.mpf(LAM) * mp.sqrt(n) / (2 * mp.mpf(a))) * 180 / mp.pi
        assert abs(oracle.two_theta(q, LAM) - float(exact)) < 1e-11


def test_triclinic_metric_inverse_against_mpmath():
    # G* against a 40-digit matrix inverse of G built from the basis vectors.
    mp.mp.dps = 40
    rng = np.random.default_rng(11)
    for _ in range(20):
        lat = np.concatenate([rng.uniform(3, 15, 3), rng.uniform(62, 118, 3)])
        res = oracle.cell(lat)
        if res is None:
            continue
        _, gs, vol = res
        a, b, c = (mp.mpf(float(x)) for x in lat[:3])
        al, be, ga = (mp.mpf(float(x)) * mp.pi / 180 for x in lat[3:])
        G = mp.matrix([[a * a, a * b * mp.cos(ga), a * c * mp.cos(be)],
                       [a * b * mp.cos(ga), b * b, b * c * mp.cos(al)],
                       [a * c * mp.cos(be), b * c * mp.cos(al), c * c]])
        Gi = G ** -1
        ref = [Gi[0, 0], Gi[1, 1], Gi[2, 2], Gi[0, 1], Gi[0, 2], Gi[1, 2]]
        scale = max(abs(float(x)) for x in ref)
        for got, want in zip(gs, ref):
            assert abs(got - float(want)) <= 1e-12 * scale
        assert vol == pytest.approx(float(mp.sqrt(mp.det(G))), rel=1e-12)


def test_invalid_cells_rejected():
    assert oracle.cell([5, 5, 5, 120, 120, 120]) is None  # flat (det 0)
    assert oracle.cell([-1, 5, 5, 90, 90, 90]) is None
    assert oracle.cell([5, 5, 5, 0, 90, 90]) is None
    assert oracle.cell([5, 5, 5, 90, 90, 180]) is None
    with pytest.raises(ValueError):
        oracle.enumerate_hkl([5, 5, 5, 90, 90, 90], LAM, 10.0, 180.0)
    with pytest.raises(ValueError):
        oracle.enumerate_hkl([5, 5, 5, 90, 90, 90], -1.0, 10.0, 90.0)


# ---- enumeration --------------------------------------------------------------

def test_cubic_counts_are_sums_of_three_squares():
    a, tmax = 5.64, 90.0
    hkl, q, tt, amb = oracle.enumerate_hkl([a, a, a, 90, 90, 90], LAM, 0.0, tmax)
    nmax = (a * 2 * math.sin(math.radians(tmax / 2)) / LAM) ** 2
    assert nmax == pytest.approx(26.761, abs=1e-3)
    want = sum(r3(n) for n in range(1, int(nmax) + 1))
    assert len(tt) == want == 586
    assert amb == 0
    n_of = (hkl.astype(np.int64) ** 2).sum(1)
    assert set(n_of) == {n for n in range(1, 27) if r3(n)}
    assert {7, 15, 23}.isdisjoint(set(n_of))  # Legendre: 4^a (8b + 7)


def test_enumeration_is_lexicographic_and_symmetric():
    lat = [4.1, 5.3, 6.7, 71.0, 103.0, 96.0]
    hkl, q, tt, _ = oracle.enumerate_hkl(lat, LAM, 10.0, 90.0)
    keys = [tuple(x) for x in hkl]
    assert keys == sorted(keys)
    assert set(keys) == {tuple(-np.array(k)) for k in keys}  # Friedel mates present
    assert np.all((tt >= 10.0) & (tt <= 90.0))


def test_enumeration_complete_against_brute_force_box():
    # A much larger box finds nothing the oracle's generous box missed.
    mp.mp.dps = 30
    lat = [3.3, 4.7, 3.9, 64.0, 117.0, 78.0]
    hkl, q, tt, _ = oracle.enumerate_hkl(lat, LAM, 5.0, 150.0)
    _, gs, _ = oracle.cell(lat)
    found = set(map(tuple, hkl))
    brute = set()
    m = 12
    for h in range(-m, m + 1):
        for k in range(-m, m + 1):
            for l in range(-m, m + 1):
                if (h, k, l) == (0, 0, 0):
                    continue
                t = oracle.two_theta(oracle.q_of(gs, h, k, l), LAM)
                if 5.0 <= t <= 150.0:
                    brute.add((h, k, l))
    assert found == brute
    assert max(abs(x) for t in found for x in t) < m  # the brute box was large enough


def test_enumeration_count_matches_sphere_volume():
    # Number of lattice points in a reciprocal shell ~ shell volume * V.
    lat = [31.0, 37.0, 44.0, 90.0, 104.0, 90.0]
    tmin, tmax = 5.0, 120.0
    hkl, q, tt, _ = oracle.enumerate_hkl(lat, LAM, tmin, tmax)
    _, _, vol = oracle.cell(lat)
    g = lambda t: 2 * math.sin(math.radians(t / 2)) / LAM
    expect = 4.0 / 3.0 * math.pi * (g(tmax) ** 3 - g(tmin) ** 3) * vol
    assert len(tt) == pytest.approx(expect, rel=2e-3)


# ---- structure factors and intensities ----------------------------------------

def test_rocksalt_closed_form():
    b = synth.rocksalt()
    r = oracle.pattern(b, 0)
    assert r.amb_bound == 0 and r.amb_gap == 0
    a = 5.64
    fa, fb = b.sf_coeff
    imax = 0.0
    rows = []
    for pt, pi, m, first in zip(r.pk_tt, r.pk_i, r.pk_mult, r.pk_first):
        h, k, l = r.hkl[r.perm[first]]
        n = int(h * h + k * k + l * l)
        assert m == r3(n)
        s2 = n / a ** 2 / 4.0
        dw = math.exp(-0.5 * s2)
        f_a = fa[8] + sum(fa[i] * math.exp(-fa[4 + i] * s2) for i in range(4))
        f_b = fb[8] + sum(fb[i] * math.exp(-fb[4 + i] * s2) for i in range(4))
        par = {x % 2 for x in (h, k, l)}
        if len(par) == 2:
            fmag = 0.0  # fcc extinction: mixed parity
        elif par == {0}:
            fmag = 4 * (f_a + f_b) * dw
        else:
            fmag = 4 * (f_a - f_b) * dw
        th = math.radians(pt / 2)
        lpv = (1 + math.cos(2 * th) ** 2) / (math.sin(th) ** 2 * math.cos(th))
        rows.append((pi, m * fmag * fmag * lpv))
        imax = max(imax, pi)
    for got, want in rows:
        if want == 0.0:
            assert got <= 1e-25 * imax
        else:
            assert got == pytest.approx(want, rel=1e-12)
    assert len(rows) == 23 and sum(1 for _, w in rows if w > 0) == 9
    assert max(r.pk_y) == 100.0
    # the strongest line of this draw is 200, the second 111
    top = np.argsort(-r.pk_i)[:2]
    assert [int((r.hkl[r.perm[r.pk_first[t]]] ** 2).sum()) for t in top] == [4, 3]


def test_bcc_extinction():
    coeff = np.array([[2.0, 1.0, 0.5, 0.2, 10.0, 3.0, 1.0, 0.5, 0.3]])
    b = cubic(3.3, [[0, 0, 0], [0.5, 0.5, 0.5]], [0, 0], coeff, bfac=0.3)
    r = oracle.pattern(b, 0)
    mx = r.inten.max()
    odd = (r.hkl.sum(1) % 2) != 0
    assert np.all(r.inten[odd] <= 1e-25 * mx)
    assert np.all(r.inten[~odd] > 1e-6 * mx)


def test_single_atom_closed_form():
    coeff = np.array([[2.0, 1.0, 0.5, 0.2, 10.0, 3.0, 1.0, 0.5, 0.3]])
    lat = [4.2, 5.1, 6.3, 80.0, 95.0, 105.0]
    bat = synth.CrystalBatch("t", np.array([lat]), np.array([0, 1], np.int64), np.zeros((1, 3)),
                             np.zeros(1, np.int32), np.array([0.7]), np.array([1.3]), coeff, LAM,
                             np.array([5.0]), np.array([120.0]))
    r = oracle.pattern(bat, 0)
    s2 = r.q / 4
    f = coeff[0, 8] + sum(coeff[0, i] * np.exp(-coeff[0, 4 + i] * s2) for i in range(4))
    th = np.radians(r.tt / 2)
    lpv = (1 + np.cos(2 * th) ** 2) / (np.sin(th) ** 2 * np.cos(th))
    want = 0.7 ** 2 * f ** 2 * np.exp(-2 * 1.3 * s2) * lpv
    np.testing.assert_allclose(r.inten, want, rtol=1e-13)
    np.testing.assert_allclose(r.fi, 0.0, atol=1e-15)


def test_two_atom_closed_form():
    coeff = np.array([[2.0, 1.0, 0.5, 0.2, 10.0, 3.0, 1.0, 0.5, 0.3],
                      [1.0, 3.0, 0.7, 0.1, 2.0, 30.0, 5.0, 1.5, 0.1]])
    lat = [4.2, 5.1, 6.3, 80.0, 95.0, 105.0]
    x = np.array([[0.11, 0.27, 0.83], [0.62, 0.04, 0.39]])
    bat = synth.CrystalBatch("t", np.array([lat]), np.array([0, 2], np.int64), x,
                             np.array([0, 1], np.int32), np.array([0.9, 0.6]), np.array([0.4, 1.7]),
                             coeff, LAM, np.array([5.0]), np.array([120.0]))
    r = oracle.pattern(bat, 0)
    s2 = r.q / 4
    w = []
    for j in range(2):
        c = coeff[j]
        f = c[8] + sum(c[i] * np.exp(-c[4 + i] * s2) for i in range(4))
        w.append([0.9, 0.6][j] * f * np.exp(-[0.4, 1.7][j] * s2))
    dphi = 2 * np.pi * (r.hkl @ (x[1] - x[0]))
    f2 = w[0] ** 2 + w[1] ** 2 + 2 * w[0] * w[1] * np.cos(dphi)
    np.testing.assert_allclose(r.fr ** 2 + r.fi ** 2, f2, rtol=1e-11, atol=1e-12 * f2.max())


def test_mpmath_brute_force_structure_factors():
    # 50-digit evaluation of the same sums for small random cells.
    mp.mp.dps = 50
    rng = np.random.default_rng(5)
    for trial in range(3):
        b = synth.random_triclinic(100 + trial, 1, len_lo=2.5, len_hi=4.0, atoms_lo=2, atoms_hi=4,
                                   pool=4, tmin=20.0, tmax=70.0)
        r = oracle.pattern(b, 0)
        assert 0 < r.n_refl <= 200
        sl = b.atoms_of(0)
        pick = rng.choice(r.n_refl, size=min(40, r.n_refl), replace=False)
        for i in pick:
            h, k, l = (int(v) for v in r.hkl[i])
            s2 = mp.mpf(r.q[i]) / 4
            re = im = mp.mpf(0)
            for x, sp, oc, bf in zip(b.frac[sl], b.species[sl], b.occ[sl], b.bfac[sl]):
                c = [mp.mpf(float(v)) for v in b.sf_coeff[sp]]
                f = c[8] + sum(c[t] * mp.exp(-c[4 + t] * s2) for t in range(4))
                w = mp.mpf(float(oc)) * f * mp.exp(-mp.mpf(float(bf)) * s2)
                ph = 2 * mp.pi * (h * mp.mpf(float(x[0])) + k * mp.mpf(float(x[1])) + l * mp.mpf(float(x[2])))
                re += w * mp.cos(ph)
                im += w * mp.sin(ph)
            scale = float(r.absw[i])
            assert abs(r.fr[i] - float(re)) <= 1e-13 * scale
            assert abs(r.fi[i] - float(im)) <= 1e-13 * scale
            want_tt = 2 * mp.asin(mp.mpf(LAM) * mp.sqrt(mp.mpf(r.q[i])) / 2) * 180 / mp.pi
            assert abs(r.tt[i] - float(want_tt)) < 1e-11


# ---- invariants ---------------------------------------------------------------

def _one(seed=7, n=12):
    return synth.random_triclinic(seed, 1, atoms_lo=n, atoms_hi=n, len_lo=4.0, len_hi=7.0)


def test_friedel_pairs_equal_intensity():
    b = _one()
    r = oracle.pattern(b, 0)
    idx = {tuple(h): i for i, h in enumerate(r.hkl)}
    for i, h in enumerate(r.hkl):
        j = idx[tuple(-h)]
        assert r.fr[j] == pytest.approx(r.fr[i], rel=1e-12, abs=1e-12 * r.absw[i])
        assert r.fi[j] == pytest.approx(-r.fi[i], rel=1e-12, abs=1e-12 * r.absw[i])
    assert np.all(r.pk_mult % 2 == 0)
    assert r.pk_mult.sum() == r.n_refl


def test_translation_permutation_and_cell_shift_invariance():
    b = _one()
    r0 = oracle.pattern(b, 0)
    sl = b.atoms_of(0)
    for mod in ("shift", "perm", "plus1"):
        b2 = b.subset([0])
        if mod == "shift":
            b2.frac = np.mod(b2.frac + np.array([0.137, 0.512, 0.901]), 1.0)
        elif mod == "perm":
            p = np.random.default_rng(3).permutation(sl.stop - sl.start)
            b2.frac, b2.species, b2.occ, b2.bfac = b2.frac[p], b2.species[p], b2.occ[p], b2.bfac[p]
        else:
            b2.frac = b2.frac + 1.0
        r = oracle.pattern(b2, 0)
        np.testing.assert_array_equal(r.pk_mult, r0.pk_mult)
        np.testing.assert_array_equal(r.pk_tt, r0.pk_tt)
        np.testing.assert_allclose(r.pk_i, r0.pk_i, rtol=1e-9, atol=1e-12 * r0.pk_i.max())


def _lattice_from_metric(G):
    a, b, c = np.sqrt(np.diag(G))
    al = math.degrees(math.acos(G[1, 2] / (b * c)))
    be = math.degrees(math.acos(G[0, 2] / (a * c)))
    ga = math.degrees(math.acos(G[0, 1] / (a * b)))
    return [a, b, c, al, be, ga]


def _metric(lat):
    a, b, c = lat[:3]
    ca, cb, cg = (math.cos(math.radians(x)) for x in lat[3:])
    return np.array([[a * a, a * b * cg, a * c * cb], [a * b * cg, b * b, b * c * ca],
                     [a * c * cb, b * c * ca, c * c]])


def _peaks_match(ra, rb, tol_pos=1e-8):
    """Peaks with I above 1e-9 of max agree in position and intensity."""
    mx = max(ra.pk_i.max(), rb.pk_i.max())
    sa = ra.pk_i > 1e-9 * mx
    sb = rb.pk_i > 1e-9 * mx
    np.testing.assert_allclose(ra.pk_tt[sa], rb.pk_tt[sb], atol=tol_pos)
    np.testing.assert_allclose(ra.pk_i[sa], rb.pk_i[sb], rtol=1e-8)


def test_unimodular_basis_change_gives_same_pattern():
    b = _one(seed=9, n=10)
    r0 = oracle.pattern(b, 0)
    M = np.array([[1, 1, 0], [0, 1, 0], [1, 0, 1]])  # det 1
    assert round(np.linalg.det(M)) == 1
    G = _metric(b.lattice[0])
    G2 = M @ G @ M.T
    b2 = b.subset([0])
    b2.lattice = np.array([_lattice_from_metric(G2)])
    b2.frac = (np.linalg.inv(M).T @ b.frac[b.atoms_of(0)].T).T
    r = oracle.pattern(b2, 0)
    np.testing.assert_array_equal(r.pk_mult, r0.pk_mult)
    np.testing.assert_allclose(r.pk_tt, r0.pk_tt, atol=1e-8)
    np.testing.assert_allclose(r.pk_i, r0.pk_i, rtol=1e-8, atol=1e-12 * r0.pk_i.max())


def test_supercell_doubles_amplitudes():
    b = _one(seed=13, n=6)
    r0 = oracle.pattern(b, 0)
    sl = b.atoms_of(0)
    x = b.frac[sl]
    b2 = b.subset([0])
    b2.lattice = b.lattice.copy()
    b2.lattice[0, 0] *= 2.0
    half = x.copy()
    half[:, 0] /= 2.0
    shifted = half.copy()
    shifted[:, 0] += 0.5
    b2.frac = np.concatenate([half, shifted])
    b2.species = np.concatenate([b.species[sl]] * 2)
    b2.occ = np.concatenate([b.occ[sl]] * 2)
    b2.bfac = np.concatenate([b.bfac[sl]] * 2)
    b2.atom_offset = np.array([0, 2 * len(x)], np.int64)
    r = oracle.pattern(b2, 0)
    odd = r.hkl[:, 0] % 2 != 0
    assert np.all(r.inten[odd] <= 1e-24 * r.inten.max())
    sub = {tuple(h): i for i, h in enumerate(r0.hkl)}
    ev = np.nonzero(~odd)[0]
    assert len(ev) == r0.n_refl
    for i in ev:
        h = r.hkl[i]
        j = sub[(h[0] // 2, h[1], h[2])]
        assert r.tt[i] == pytest.approx(r0.tt[j], abs=1e-9)
        assert r.inten[i] == pytest.approx(4.0 * r0.inten[j], rel=1e-9, abs=1e-12 * r.inten.max())


# ---- sort and merge -----------------------------------------------------------

def test_anchor_merge_rule():
    tol = 1e-5
    t = np.array([10.0, 10.0 + 0.6 * tol, 10.0 + 1.2 * tol, 10.0 + 1.3 * tol, 10.0 + 5 * tol])
    i = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    pt, pi, pm, pf, amb = oracle.merge(t, i, tol)
    # anchor rule: {0,1} {2,3} {4}; single linkage would give {0..3} {4}
    np.testing.assert_array_equal(pm, [2, 2, 1])
    np.testing.assert_array_equal(pf, [0, 2, 4])
    np.testing.assert_array_equal(pt, [t[0], t[2], t[4]])  # anchor, not mean
    np.testing.assert_array_equal(pi, [3.0, 12.0, 16.0])
    assert amb == 0
    # a difference exactly at the tolerance opens a new peak (strict "<")
    pt, pi, pm, pf, amb = oracle.merge(np.array([1.0, 1.5]), np.array([1.0, 1.0]), 0.5)
    np.testing.assert_array_equal(pm, [1, 1])
    assert amb == 1
    assert oracle.merge(np.zeros(0), np.zeros(0), tol)[0].size == 0


def test_sort_breaks_ties_by_hkl():
    tt = np.array([20.0, 10.0, 20.0, 10.0, 15.0])
    hkl = np.array([[1, 0, 0], [0, 0, 1], [-1, 0, 0], [0, 0, -1], [0, 1, 0]], np.int32)
    perm = oracle.sort_order(tt, hkl)
    np.testing.assert_array_equal(perm, [3, 1, 4, 2, 0])


def test_threshold_and_scaling():
    b = synth.rocksalt()
    r = oracle.pattern(b, 0, threshold=0.05)
    full = oracle.pattern(b, 0)
    keep = full.pk_i >= 0.05 * full.pk_i.max()
    np.testing.assert_array_equal(r.pk_tt, full.pk_tt[keep])
    np.testing.assert_allclose(r.pk_y, 100 * full.pk_i[keep] / full.pk_i.max(), rtol=1e-15)


def test_empty_and_atomless_crystals():
    coeff = np.array([[2.0, 1.0, 0.5, 0.2, 10.0, 3.0, 1.0, 0.5, 0.3]])
    # no atoms: every intensity 0, scaled 0
    b = synth.CrystalBatch("t", np.array([[4.0, 4.0, 4.0, 90, 90, 90]]), np.array([0, 0], np.int64),
                           np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros(0), np.zeros(0), coeff,
                           LAM, np.array([10.0]), np.array([90.0]))
    r = oracle.pattern(b, 0)
    assert r.n_refl > 0 and np.all(r.inten == 0) and np.all(r.pk_y == 0)
    # range below the first reflection: nothing at all
    b.two_theta_max = np.array([12.0])
    r = oracle.pattern(b, 0)
    assert r.n_refl == 0 and r.pk_tt.size == 0


# ---- broadening ----------------------------------------------------------------

def test_broadening_single_line_and_area():
    t0, dt, n, sig, win = 10.0, 0.02, 4001, 0.1, 8.0
    y = oracle.broaden(np.array([50.013]), np.array([3.0]), t0, dt, n, sig, win)
    x = t0 + dt * np.arange(n)
    want = 3.0 * np.exp(-(x - 50.013) ** 2 / (2 * sig ** 2)) / (sig * math.sqrt(2 * math.pi))
    want[np.abs(x - 50.013) > win * sig] = 0.0
    np.testing.assert_allclose(y, want, rtol=1e-13, atol=1e-300)
    assert y.sum() * dt == pytest.approx(3.0, rel=1e-9)  # unit-area kernel
    assert np.count_nonzero(y) == 80 or np.count_nonzero(y) == 81
    # outside the grid, nothing
    assert not oracle.broaden(np.array([100.0]), np.array([1.0]), t0, dt, n, sig, win).any()


def test_range_bounds_are_inclusive():
    # A reflection whose 2theta equals a bound exactly is kept at both ends.
    a = 4.0
    _, gs, _ = oracle.cell([a, a, a, 90, 90, 90])
    t100 = oracle.two_theta(oracle.q_of(gs, 1, 0, 0), LAM)
    t111 = oracle.two_theta(oracle.q_of(gs, 1, 1, 1), LAM)
    hkl, q, tt, amb = oracle.enumerate_hkl([a, a, a, 90, 90, 90], LAM, t100, t111)
    n = (hkl.astype(int) ** 2).sum(1)
    assert sorted(set(n)) == [1, 2, 3]
    assert len(tt) == 6 + 12 + 8
    assert amb == 6 + 8  # the bound-touching reflections are flagged as ambiguous
