"""Pins of the oracle's augmentation functions (preferred orientation and
noise): closed forms, the March-Dollase normalisation over the sphere, the
published SplitMix64 sequence and the moments of the normal variates."""

import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cubic_gs(a=4.0):
    return np.array([1 / a**2, 1 / a**2, 1 / a**2, 0.0, 0.0, 0.0])


@pytest.mark.parametrize("r", [0.3, 0.7, 1.0, 1.6])
def test_march_dollase_closed_forms(r):
    gs = cubic_gs()
    # parallel: P = r^-3; perpendicular: P = r^(3/2); r = 1: no texture
    assert oracle.march_dollase(gs, 2, 0, 0, [1, 0, 0], r) == pytest.approx(r**-3, rel=1e-14)
    assert oracle.march_dollase(gs, 0, 3, 0, [1, 0, 0], r) == pytest.approx(r**1.5, rel=1e-14)
    assert oracle.march_dollase(gs, 1, 1, 0, [1, 0, 0], 1.0) == pytest.approx(1.0, rel=1e-14)
    # 45 degrees in a cubic cell: cos^2 = 1/2
    assert oracle.march_dollase(gs, 1, 1, 0, [1, 0, 0], r) == pytest.approx((0.5 * r * r + 0.5 / r) ** -1.5,
                                                                           rel=1e-14)
    # antiparallel equals parallel; the factor depends on direction only
    assert oracle.march_dollase(gs, -2, 0, 0, [1, 0, 0], r) == pytest.approx(r**-3, rel=1e-14)
    assert oracle.march_dollase(gs, 1, 0, 0, [5, 0, 0], r) == pytest.approx(r**-3, rel=1e-14)


def test_march_dollase_metric():
    """In a non-orthogonal cell the angle comes from G*: for a hexagonal cell
    (gamma = 120) the reciprocal axes a* and b* meet at 60 degrees."""
    _, gs, _ = oracle.cell([3.0, 3.0, 5.0, 90.0, 90.0, 120.0])
    r = 0.6
    want = (r * r * 0.25 + 0.75 / r) ** -1.5
    assert oracle.march_dollase(gs, 0, 1, 0, [1, 0, 0], r) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("r", [0.5, 1.4])
def test_march_dollase_is_normalised(r):
    """The March-Dollase distribution averages to 1 over the sphere; the
    lattice directions of a cubic cell inside a large ball sample it evenly."""
    gs = cubic_gs()
    hp = np.array([1.0, 2.0, 2.0])
    n = 24
    vals = [oracle.march_dollase(gs, h, k, l, hp, r)
            for h in range(-n, n + 1) for k in range(-n, n + 1) for l in range(-n, n + 1)
            if 0 < h * h + k * k + l * l <= n * n]
    assert np.mean(vals) == pytest.approx(1.0, abs=3e-3)


def test_splitmix64_published_sequence():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if not l.startswith("#")]
    for j, v in rows:
        assert oracle.splitmix64(0, int(j)) == int(v, 16)


def test_gauss_moments_and_determinism():
    z = np.array([oracle.gauss(12345, n) for n in range(200000)])
    assert abs(z.mean()) < 0.01
    assert z.var() == pytest.approx(1.0, abs=0.01)
    assert np.mean(np.abs(z) < 1.0) == pytest.approx(0.6827, abs=0.005)
    # the fourth moment of a standard normal is 3
    assert np.mean(z**4) == pytest.approx(3.0, abs=0.06)
    assert oracle.gauss(12345, 7) == z[7] and oracle.gauss(12346, 7) != z[7]


def test_noise_definition():
    y = np.abs(np.random.default_rng(3).normal(size=(3, 50))) * 10
    out = oracle.noise(y, 99, 0.2, 0.05)
    z = np.array([oracle.gauss(99, i) for i in range(y.size)]).reshape(y.shape)
    np.testing.assert_allclose(out, y + (0.2 * np.sqrt(y) + 0.05) * z, rtol=1e-15, atol=0)
    np.testing.assert_array_equal(oracle.noise(y, 99, 0.0, 0.0), y)


def test_noise_moments():
    """Noise added to flat rows: zero mean and the variance of the stated
    model, (rel sqrt(max(y, 0)) + abs)^2, per row, with the counting term
    growing with the level and absent below zero, and no correlation between
    rows.  Pins the definition by its statistics rather than its formula."""
    n = 100000
    levels = np.array([25.0, 4.0, -3.0, 0.0])
    rel, abs_ = 0.1, 0.02
    y = np.repeat(levels[:, None], n, axis=1)
    e = oracle.noise(y, 2024, rel, abs_) - y
    for row, v in enumerate(levels):
        sd = rel * np.sqrt(max(v, 0.0)) + abs_
        assert abs(e[row].mean()) <= 5 * sd / np.sqrt(n), row
        assert e[row].var() == pytest.approx(sd * sd, rel=0.02), row
        # fourth moment of a normal: 3 sd^4
        assert np.mean(e[row] ** 4) == pytest.approx(3 * sd ** 4, rel=0.06), row
    # the -3 and 0 rows both carry only the flat term
    assert e[2].std() == pytest.approx(abs_, rel=0.02) and e[3].std() == pytest.approx(abs_, rel=0.02)
    z = e / (rel * np.sqrt(np.maximum(levels, 0.0)) + abs_)[:, None]
    assert abs(np.corrcoef(z[0], z[1])[0, 1]) < 0.02


def test_caglioti_reduces_to_constant_width():
    rng = np.random.default_rng(8)
    tt = np.sort(rng.uniform(15, 80, 40))
    inten = rng.uniform(0.5, 5, 40)
    W = 0.04
    sigma = np.sqrt(W) / (2 * np.sqrt(2 * np.log(2)))
    a = oracle.broaden_caglioti(tt, inten, 10.0, 0.01, 8001, 0.0, 0.0, W, 8.0)
    b = oracle.broaden(tt, inten, 10.0, 0.01, 8001, sigma, 8.0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13 * b.max())


@pytest.mark.parametrize("tt0", [20.0, 70.0, 120.0])
def test_caglioti_width_and_area(tt0):
    """A single line: unit area times its intensity, and the full width at
    half maximum of the formula (found on a fine grid)."""
    U, V, W = 0.02, -0.01, 0.005
    th = np.radians(tt0 / 2)
    fwhm = np.sqrt(U * np.tan(th) ** 2 + V * np.tan(th) + W)
    dt = 1e-4
    n = int(2.0 / dt) + 1
    t0 = tt0 - 1.0
    y = oracle.broaden_caglioti([tt0], [3.0], t0, dt, n, U, V, W, 8.0)
    assert np.sum(y) * dt == pytest.approx(3.0, rel=1e-6)
    above = np.nonzero(y >= 0.5 * y.max())[0]
    assert (above[-1] - above[0]) * dt == pytest.approx(fwhm, abs=2 * dt)


def test_caglioti_skips_nonpositive_widths():
    y = oracle.broaden_caglioti([30.0, 60.0], [1.0, 1.0], 10.0, 0.01, 8001, 0.0, 0.0, -0.1, 8.0)
    assert not y.any()


def test_pseudo_voigt_lorentzian_area_is_truncated_arctangent():
    """eta = 1: a unit-area Lorentzian of FWHM Gam cut at |d| <= h has area
    (2 / pi) atan(2 h / Gam); times the intensity, on a fine grid."""
    W, window = 0.01, 8.0
    gam = np.sqrt(W)
    h = window * gam / (2 * np.sqrt(2 * np.log(2)))
    dt = 1e-5
    n = int(2 * 1.0 / dt) + 1
    y = oracle.broaden_caglioti([40.0], [2.0], 39.0, dt, n, 0.0, 0.0, W, window, eta=1.0)
    # the rectangle sum misses at most one grid step of the cut-off tail on
    # each side: 2 dt I L(h), with L(h) = (2 / (pi Gam)) / (1 + (2 h / Gam)^2)
    edge = 2 * dt * 2.0 * (2 / (np.pi * gam)) / (1 + (2 * h / gam) ** 2)
    assert abs(np.sum(y) * dt - 2.0 * (2 / np.pi) * np.arctan(2 * h / gam)) <= edge + 1e-9


@pytest.mark.parametrize("eta", [0.0, 0.3, 1.0])
def test_pseudo_voigt_peak_value_and_half_maximum(eta):
    """At the line centre the profile is eta 2/(pi Gam) + (1 - eta)/(sigma
    sqrt(2 pi)); at d = +-Gam/2 both components, hence the sum, are halved."""
    gam, dt = 0.1, 0.01  # Gam / 2 = 5 grid steps
    sigma = gam / (2 * np.sqrt(2 * np.log(2)))
    y = oracle.broaden_caglioti([30.0], [1.5], 29.0, dt, 201, 0.0, 0.0, gam * gam, 30.0, eta=eta)
    c = 100  # x = 30.0
    peak = 1.5 * (eta * 2 / (np.pi * gam) + (1 - eta) / (sigma * np.sqrt(2 * np.pi)))
    assert y[c] == pytest.approx(peak, rel=1e-12)
    assert y[c - 5] == pytest.approx(0.5 * peak, rel=1e-9) and y[c + 5] == pytest.approx(0.5 * peak, rel=1e-9)


def test_pseudo_voigt_is_linear_in_eta():
    rng = np.random.default_rng(9)
    tt = np.sort(rng.uniform(15, 80, 30))
    inten = rng.uniform(0.5, 5, 30)
    args = (tt, inten, 10.0, 0.01, 8001, 0.02, -0.005, 0.004, 12.0)
    g, l = oracle.broaden_caglioti(*args, eta=0.0), oracle.broaden_caglioti(*args, eta=1.0)
    m = oracle.broaden_caglioti(*args, eta=0.25)
    np.testing.assert_allclose(m, 0.25 * l + 0.75 * g, rtol=1e-12, atol=1e-14 * g.max())
