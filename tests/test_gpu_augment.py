"""Preferred orientation and noise on the GPU against the oracle's
definitions, element by element, and a textured pattern end to end."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.test_gpu_forward import ragged_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


def texture(n_c, seed=5):
    rng = np.random.default_rng(seed)
    hp = rng.normal(size=(n_c, 3))
    r = rng.uniform(0.4, 1.8, n_c)
    return hp, r


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_march_dollase_per_reflection(precision):
    from paper_2602_11709_amd.api import XrdBatch
    b = ragged_batch()
    hp, r = texture(b.n_crystals)
    r[2] = 1.0          # random powder: unchanged
    r[4] = -1.0         # switched off
    hp[5] = 0.0         # no direction: switched off
    hp[0] = [0.0, 0.0, 1.0]  # an integer direction
    xb = XrdBatch(b, precision=precision)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    before = I.clone()
    xb.preferred_orientation(refl, I, hp, r)
    torch.cuda.synchronize()
    ro, _ = xb.read_counts(refl)
    n = int(ro[-1])
    I0, I1 = before[:n].cpu().numpy(), I[:n].cpu().numpy()
    hkl = np.stack([refl.h[:n].cpu().numpy(), refl.k[:n].cpu().numpy(), refl.l[:n].cpu().numpy()], axis=1)
    for c in range(b.n_crystals):
        sl = slice(int(ro[c]), int(ro[c + 1]))
        if sl.stop == sl.start:
            continue
        if c in (2, 4, 5):
            np.testing.assert_allclose(I1[sl], I0[sl], rtol=1e-15 if c == 2 else 0)
            continue
        _, gs, _ = oracle.cell(b.lattice[c])
        P = np.array([oracle.march_dollase(gs, *m, hp[c], r[c]) for m in hkl[sl]])
        np.testing.assert_allclose(I1[sl], I0[sl] * P, rtol=1e-12, err_msg=f"crystal {c}")


def test_textured_pattern_end_to_end():
    """Texture applied before the merge: every peak carries the sum of its
    members' textured intensities."""
    from paper_2602_11709_amd.api import XrdBatch
    b = synth.random_triclinic(91, 8, atoms_hi=30)
    hp, r = texture(b.n_crystals, 6)
    xb = XrdBatch(b, precision="fp64")
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    xb.preferred_orientation(refl, I, hp, r)
    pk = xb.merge(refl, I)
    ro, po = xb.read_counts(refl, pk)
    pi = pk.intensity[:int(po[-1])].cpu().numpy()
    for c in range(b.n_crystals):
        o = oracle.pattern(b, c)
        _, gs, _ = oracle.cell(b.lattice[c])
        P = np.array([oracle.march_dollase(gs, *m, hp[c], r[c]) for m in o.hkl])
        want = np.array([np.sum((o.inten * P)[o.perm[f:f + m]]) for f, m in zip(o.pk_first, o.pk_mult)])
        got = pi[int(po[c]):int(po[c + 1])]
        assert len(got) == len(want)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12 * max(want.max(), 1e-300))


def test_noise_matches_definition_and_seed():
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = synth.random_triclinic(92, 5, atoms_hi=30)
    grid = Grid(10.0, 0.02, 4001, 0.1, 8.0)
    xb = XrdBatch(b, precision="mixed", grid_capacity=grid.n_points)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    y = xb.pattern_forward(refl, I, grid)
    torch.cuda.synchronize()
    y0 = y.cpu().numpy().copy()
    seed = 0xDEADBEEF12345
    xb.noise(y, seed, 0.05, 0.01)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    want = oracle.noise(y0, seed, 0.05, 0.01)
    scale = 0.05 * np.sqrt(np.maximum(y0, 0)) + 0.01
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * float(np.max(np.abs(want))))
    # the added noise has unit-normal shape once divided by its scale
    z = (got - y0) / scale
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    # same seed, same noise; another seed, other noise
    y2 = torch.as_tensor(y0).cuda()
    xb.noise(y2, seed, 0.05, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), got)
    y3 = torch.as_tensor(y0).cuda()
    xb.noise(y3, seed + 1, 0.05, 0.01)
    torch.cuda.synchronize()
    assert not np.array_equal(y3.cpu().numpy(), got)


@pytest.mark.parametrize("precision,friedel,uvw,eta", [
    ("mixed", True, (0.03, -0.01, 0.004), 0.0), ("fp64", False, (0.03, -0.01, 0.004), 0.0),
    # FWHM^2 <= 0 below 2theta ~ 11.4 deg: those lines add nothing
    ("fp64", True, (0.05, 0.0, -0.0005), 0.0),
    # widest line at the quadratic's vertex (tan theta = 0.75, 2theta ~ 73.7 deg), not at an end
    ("mixed", False, (-0.02, 0.03, 0.002), 0.0),
    # pseudo-Voigt profiles
    ("mixed", True, (0.03, -0.01, 0.004), 0.4), ("fp64", True, (0.03, -0.01, 0.004), 1.0)])
def test_caglioti_pattern(precision, friedel, uvw, eta):
    """Widths growing with angle, against the oracle's broadening of the GPU's
    own reflections and intensities, on crystals of every sort size (the
    largest sorted in global memory) and a grid cut at both ends."""
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = ragged_batch()
    grid = Grid(12.0, 0.017, 4501, 1.0, 8.0)
    U, V, W = uvw
    xb = XrdBatch(b, precision=precision, friedel=friedel)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    y = xb.pattern_caglioti(refl, I, grid, U, V, W, eta=eta)
    torch.cuda.synchronize()
    ro, _ = xb.read_counts(refl)
    n = int(ro[-1])
    tt, Ih, yh = refl.two_theta[:n].cpu().numpy(), I[:n].cpu().numpy(), y.cpu().numpy()
    for c in range(b.n_crystals):
        sl = slice(int(ro[c]), int(ro[c + 1]))
        want = oracle.broaden_caglioti(tt[sl], Ih[sl], grid.t0, grid.dt, grid.n_points, U, V, W, grid.window_sigmas,
                                       eta=eta)
        err = np.max(np.abs(yh[c] - want)) / max(np.max(np.abs(want)), 1e-300)
        tol = 1e-12 if precision == "fp64" else 1e-5  # single-precision exponentials under mixed
        assert err <= tol, f"crystal {c}: {err:.3e}"
    # repeat: bit for bit
    y2 = xb.pattern_caglioti(refl, I, grid, U, V, W, eta=eta)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)


def test_augmentations_full_workload():
    """The 1024-crystal workload the benchmark times: Caglioti / pseudo-Voigt
    patterns on sampled crystals, March-Dollase factors on sampled
    reflections and noise on sampled grid points, each against the oracle."""
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = synth.triclinic_1024()
    grid = Grid(10.0, 0.02, 4001, 0.1, 8.0)
    xb = XrdBatch(b, precision="mixed", friedel=True, grid_capacity=grid.n_points)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    torch.cuda.synchronize()
    ro, _ = xb.read_counts(refl)
    n = int(ro[-1])
    tt, I0 = refl.two_theta[:n].cpu().numpy(), I[:n].cpu().numpy().copy()
    rng = np.random.default_rng(21)
    crystals = rng.choice(b.n_crystals, 12, replace=False)
    for eta in (0.0, 0.5):
        y = xb.pattern_caglioti(refl, I, grid, 0.02, -0.005, 0.004, eta=eta)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        for c in crystals:
            sl = slice(int(ro[c]), int(ro[c + 1]))
            want = oracle.broaden_caglioti(tt[sl], I0[sl], grid.t0, grid.dt, grid.n_points, 0.02, -0.005, 0.004,
                                           grid.window_sigmas, eta=eta)
            err = np.max(np.abs(yh[c] - want)) / max(np.max(np.abs(want)), 1e-300)
            assert err <= 1e-5, f"eta {eta} crystal {c}: {err:.3e}"
    hp, r = texture(b.n_crystals, seed=6)
    xb.preferred_orientation(refl, I, hp, r)
    torch.cuda.synchronize()
    I1 = I[:n].cpu().numpy()
    hkl = np.stack([t[:n].cpu().numpy() for t in (refl.h, refl.k, refl.l)], axis=1)
    crystal_of = np.searchsorted(ro, np.arange(n), side="right") - 1
    for i in rng.choice(n, 4000, replace=False):
        c = crystal_of[i]
        _, gs, _ = oracle.cell(b.lattice[c])
        want = I0[i] * oracle.march_dollase(gs, *hkl[i], hp[c], r[c])
        assert I1[i] == pytest.approx(want, rel=1e-12), f"reflection {i} of crystal {c}"
    y0 = yh.copy()
    seed = 987654321
    xb.noise(y, seed, 0.05, 0.01)
    torch.cuda.synchronize()
    got = y.cpu().numpy().ravel()
    flat = y0.ravel()
    for g in rng.choice(flat.size, 4000, replace=False):
        want = flat[g] + (0.05 * np.sqrt(max(flat[g], 0.0)) + 0.01) * oracle.gauss(seed, int(g))
        assert got[g] == pytest.approx(want, rel=1e-12, abs=1e-12), f"point {g}"
