"""Element-by-element comparison of the GPU pipeline with the FP64 oracle.

Tolerances follow from the arithmetic of each path:

* reflections (h, k, l), their sorted order and the peak partition (first
  member, member count) are integers: exact, the order and partition against
  the oracle's sort and merge applied to the GPU's own 2theta values, and the
  partition also against the oracle's own 2theta wherever the oracle counted
  no ambiguous comparison (a 2theta difference within 1e-9 deg of the
  tolerance, or a 2theta within 1e-9 deg of a range bound);
* q: both sides evaluate the same double expression from G*, which they
  obtain by different formulas (reciprocal cell vs. cofactor inverse), so
  they differ by a few ulp: relative 1e-13;
* 2theta: the merge keys; 1e-9 deg (the bar for "exact positions"), and a
  peak's position is the 2theta of its first member;
* structure factors: the error of a sum is bounded by the sum of the
  magnitudes of its terms, sum_j |w_j| (the oracle reports it as ``absw``).
  Double path: each term carries a few ulp (sincos, exp, the phase), so
  |dF| <= 1e-12 sum|w|.  Mixed path: each term carries the float error of
  v_sin/v_cos (measured 1.2e-7 absolute on gfx950), of exp2 and of the
  weight (~2e-7 relative), and float sums of at most 64 atoms add up to
  63 * 2^-24 of sum|w|; the compensated outer sum adds nothing at this
  level, so |dF| <= 4.5e-6 sum|w|;
* intensities I = |F|^2 LP: |dI| <= LP (2 |F| dF + dF^2) + 1e-12 I, and for
  merged peaks the sum of the member bounds.  On top, the headline bar:
  peaks with I >= 1e-3 of the crystal's strongest peak agree within 1e-4
  relative.
"""

from __future__ import annotations

import numpy as np

import oracle

F_REL = {"fp64": 1e-12, "mixed": 4.5e-6}


def compare_crystal(res, c, orc, precision, label="", tol=1e-5):
    """Assert parity of crystal ``c`` of a PatternResult with an OracleCrystal.
    Returns a dict of error statistics."""
    rs, ps = res.crystal(c)
    tag = f"{label} crystal {c}"
    n = rs.stop - rs.start
    assert n == orc.n_refl, f"{tag}: {n} reflections vs oracle {orc.n_refl}"
    stats = {"n_refl": n, "n_peaks": ps.stop - ps.start}
    if n == 0:
        assert ps.stop == ps.start
        return stats
    np.testing.assert_array_equal(res.hkl[rs], orc.hkl, err_msg=f"{tag}: hkl list")
    np.testing.assert_allclose(res.q[rs], orc.q, rtol=1e-13, atol=0, err_msg=f"{tag}: q")
    assert np.max(np.abs(res.two_theta[rs] - orc.tt)) <= 1e-9, f"{tag}: 2theta"
    np.testing.assert_allclose(res.lp[rs], orc.lp, rtol=1e-12, err_msg=f"{tag}: LP")

    dF = F_REL[precision] * orc.absw
    eA = np.abs(res.A[rs] - orc.fr)
    eB = np.abs(res.B[rs] - orc.fi)
    assert np.all(eA <= dF + 1e-300), f"{tag}: Re F max err/bound {np.max(eA / np.maximum(dF, 1e-300)):.3g}"
    assert np.all(eB <= dF + 1e-300), f"{tag}: Im F max err/bound {np.max(eB / np.maximum(dF, 1e-300)):.3g}"
    fabs = np.sqrt(orc.fr ** 2 + orc.fi ** 2)
    dI = orc.lp * (2 * fabs * dF + dF * dF) + 1e-12 * orc.inten
    eI = np.abs(res.I[rs] - orc.inten)
    assert np.all(eI <= dI + 1e-300), f"{tag}: I max err/bound {np.max(eI / np.maximum(dI, 1e-300)):.3g}"
    stats["F_err_over_absw"] = float(np.max(np.maximum(eA, eB) / np.maximum(orc.absw, 1e-300)))

    # peaks.  The merge is checked exactly by running the oracle's sort and
    # merge on the GPU's own 2theta values (identical inputs must give an
    # identical permutation and partition); the GPU's 2theta is within 1e-9
    # deg of the oracle's, so the partition from the oracle's own 2theta agrees
    # too unless a comparison there was ambiguous (|difference - tol| < 1e-9).
    m = ps.stop - ps.start
    tt_g = res.two_theta[rs]
    perm = res.perm[rs] - rs.start
    np.testing.assert_array_equal(perm, oracle.sort_order(tt_g, res.hkl[rs]), err_msg=f"{tag}: sorted order")
    g_tt, g_i, g_m, g_f, _ = oracle.merge(tt_g[perm], orc.inten[perm], tol)
    assert m == len(g_tt), f"{tag}: {m} peaks vs {len(g_tt)} from the oracle's merge of the GPU 2theta"
    first = res.pk_first[ps] - rs.start
    np.testing.assert_array_equal(first, g_f, err_msg=f"{tag}: peak first member")
    np.testing.assert_array_equal(res.pk_mult[ps], g_m, err_msg=f"{tag}: multiplicity")
    np.testing.assert_array_equal(res.pk_two_theta[ps], g_tt, err_msg=f"{tag}: peak 2theta is the anchor's")
    if orc.amb_gap == 0 and orc.amb_bound == 0:
        np.testing.assert_array_equal(first, orc.pk_first, err_msg=f"{tag}: partition vs oracle 2theta")
        assert np.max(np.abs(res.pk_two_theta[ps] - orc.pk_tt)) <= 1e-9, f"{tag}: peak 2theta"
    stats["ambiguous"] = int(orc.amb_gap + orc.amb_bound)
    # sorted order is ascending 2theta
    assert np.all(np.diff(tt_g[perm]) >= 0), f"{tag}: perm not ascending"
    pk_bound = np.add.reduceat(dI[perm], g_f) if m else np.zeros(0)
    ePk = np.abs(res.pk_intensity[ps] - g_i)
    assert np.all(ePk <= pk_bound + 1e-300), f"{tag}: peak I max err/bound {np.max(ePk / np.maximum(pk_bound, 1e-300)):.3g}"
    imax = g_i.max() if m else 0.0
    if imax > 0:
        strong = g_i >= 1e-3 * imax
        rel = ePk[strong] / g_i[strong]
        assert np.all(rel <= 1e-4), f"{tag}: strong-peak relative error {rel.max():.3g}"
        stats["peak_rel_err"] = float(rel.max())
        stats["weak_abs_err_over_max"] = float(np.max(ePk[~strong]) / imax) if np.any(~strong) else 0.0
        # y = 100 I / I_max: error from I and from I_max
        jmax = int(np.argmax(g_i))
        g_y = 100.0 * g_i / imax
        y_bound = 100.0 * (pk_bound + g_i * pk_bound[jmax] / imax) / imax + 1e-12 * g_y
        eY = np.abs(res.pk_scaled[ps] - g_y)
        assert np.all(eY <= y_bound), f"{tag}: scaled max err/bound {np.max(eY / np.maximum(y_bound, 1e-300)):.3g}"
    else:
        assert np.all(res.pk_scaled[ps] == 0)
    return stats


def compare_batch(res, batch, orcs, precision, label=""):
    worst = {"ambiguous": 0}
    for c in range(batch.n_crystals):
        st = compare_crystal(res, c, orcs[c], precision, label, tol=batch.merge_tol)
        for k, v in st.items():
            if isinstance(v, float):
                worst[k] = max(worst.get(k, 0.0), v)
        worst["ambiguous"] += st.get("ambiguous", 0)
    return worst


def compare_crystal_sampled(res, c, batch, precision, rng, n_sample=400, n_strong=60, label=""):
    """Parity of crystal ``c`` of a PatternResult when the oracle cannot sum
    every structure factor in seconds: the reflection list and the peak
    partition exactly (partition against the oracle's sort and merge of the
    GPU's own 2theta, and against the oracle's 2theta away from ambiguous
    comparisons), structure factors on ``n_sample`` random reflections and
    intensities of ``n_strong`` random strong peaks summed from the oracle's
    member structure factors."""
    tag = f"{label} crystal {c}"
    rs, ps = res.crystal(c)
    sl = batch.atoms_of(c)
    hkl, q, tt, amb = oracle.enumerate_hkl(batch.lattice[c], batch.wavelength, float(batch.two_theta_min[c]),
                                           float(batch.two_theta_max[c]))
    n = len(tt)
    assert rs.stop - rs.start == n, f"{tag}: {rs.stop - rs.start} reflections vs oracle {n}"
    np.testing.assert_array_equal(res.hkl[rs], hkl, err_msg=f"{tag}: hkl list")
    assert np.max(np.abs(res.two_theta[rs] - tt)) <= 1e-9, f"{tag}: 2theta"
    tt_g = res.two_theta[rs]
    hkl_g = res.hkl[rs]
    perm = res.perm[rs] - rs.start
    np.testing.assert_array_equal(perm, oracle.sort_order(tt_g, hkl_g), err_msg=f"{tag}: sorted order")
    g_tt, _, g_m, g_f, _ = oracle.merge(tt_g[perm], np.zeros(n), batch.merge_tol)
    first = res.pk_first[ps] - rs.start
    np.testing.assert_array_equal(res.pk_mult[ps], g_m, err_msg=f"{tag}: multiplicity")
    np.testing.assert_array_equal(first, g_f, err_msg=f"{tag}: peak first member")
    np.testing.assert_array_equal(res.pk_two_theta[ps], g_tt, err_msg=f"{tag}: peak 2theta")
    po = oracle.sort_order(tt, hkl)
    _, _, _, o_f, amb_gap = oracle.merge(tt[po], np.zeros(n), batch.merge_tol)
    if amb_gap == 0 and amb == 0:
        np.testing.assert_array_equal(first, o_f, err_msg=f"{tag}: partition vs oracle 2theta")
    else:
        differ = len(set(first.tolist()) ^ set(o_f.tolist()))
        assert differ <= 2 * (amb_gap + amb), f"{tag}: partition differs beyond the ambiguous comparisons"
    args = (batch.frac[sl], batch.species[sl], batch.occ[sl], batch.bfac[sl], batch.sf_coeff)
    pick = rng.choice(n, size=min(n_sample, n), replace=False)
    fr, fi, aw = oracle.structure_factors(hkl[pick], q[pick], *args)
    bound = F_REL[precision] * aw
    eA = np.abs(res.A[rs][pick] - fr)
    eB = np.abs(res.B[rs][pick] - fi)
    assert np.all(eA <= bound) and np.all(eB <= bound), f"{tag}: sampled F"
    stats = {"n_refl": n, "F_err_over_absw": float(np.max(np.maximum(eA, eB) / aw))}
    pki = res.pk_intensity[ps]
    if len(pki) and pki.max() > 0:
        strong = np.nonzero(pki >= 1e-3 * pki.max())[0]
        worst = 0.0
        for p in rng.choice(strong, size=min(n_strong, len(strong)), replace=False):
            mem = perm[first[p]: first[p] + res.pk_mult[ps][p]]
            fr, fi, _ = oracle.structure_factors(hkl[mem], q[mem], *args)
            lpv = np.array([oracle.lp(t) for t in tt[mem]])
            want = float(((fr * fr + fi * fi) * lpv).sum())
            worst = max(worst, abs(pki[p] - want) / want)
        assert worst <= (1e-4 if precision == "mixed" else 1e-10), f"{tag}: strong peaks {worst:.3g}"
        stats["peak_rel_err"] = worst
    return stats
