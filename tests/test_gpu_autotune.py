"""Tile shape and split-K autotuner of the structure-factor launches: every
tile shape (1, 2, 4 reflections per lane) matches the FP64 oracle and the
others to rounding, forward and adjoint; after tuning, the forward pipeline
still matches the oracle, the structure factors agree with the defaults to
rounding, and the pattern gradients with the untuned ones."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.parity import compare_batch
from tests.test_gpu_forward import ragged_batch

pytestmark = pytest.mark.gpu

CANDIDATES = {8, 16, 24, 32, 48, 64, 96, 128, 256, 512, 2**31 - 1}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tuned_forward_matches_oracle(precision):
    from paper_2602_11709_amd.api import simulate
    b = ragged_batch()
    res = simulate(b, precision=precision, autotune=True)
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, precision, "tuned ragged")
    assert worst["ambiguous"] == 0
    print(precision, worst, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tuning_changes_only_rounding(precision):
    """Structure factors and pattern gradients before and after tuning, on a
    batch whose crystals range from 1 to 200 atoms (both sides of every
    candidate split)."""
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = synth.random_triclinic(57, 48, atoms_lo=1, atoms_hi=200)
    grid = Grid(10.0, 0.02, 4001, 0.1, 8.0)
    xb = XrdBatch(b, precision=precision, keep_sf_derivs=True, grid_capacity=grid.n_points)
    refl = xb.enumerate()
    dy = torch.randn(b.n_crystals, grid.n_points, dtype=torch.float64,
                     generator=torch.Generator().manual_seed(5)).cuda()

    def run():
        A, B, I = xb.structure_factors(refl)
        xb.pattern_forward(refl, I, grid)
        g = xb.pattern_backward(refl, grid, dy)
        torch.cuda.synchronize()
        return [t.double().cpu().numpy().copy() for t in (A, B, I)], [t.cpu().numpy().copy() for t in g]

    (A0, B0, I0), g0 = run()
    fwd, bw, _ = xb.autotune(refl)
    print(precision, "chosen splits", fwd, bw, "reflections per lane", xb.sf_rpt, flush=True)
    assert fwd in CANDIDATES and bw in CANDIDATES and xb.sf_rpt in (1, 2, 4)
    (A1, B1, I1), g1 = run()
    n = int(xb.read_counts(refl)[0][-1])
    F0 = np.hypot(A0[:n], B0[:n])
    scale = max(F0.max(), 1e-300)
    tol = 1e-5 if precision == "mixed" else 1e-12
    assert np.max(np.abs(A1[:n] - A0[:n])) <= tol * scale
    assert np.max(np.abs(B1[:n] - B0[:n])) <= tol * scale
    for name, a, c in zip(("dfrac", "dbfac", "dlat"), g0, g1):
        err = np.max(np.abs(c - a)) / max(np.max(np.abs(a)), 1e-300)
        assert err <= (1e-4 if precision == "mixed" else 1e-10), f"{name}: {err:.3e}"
    # runs with the tuned tables repeat bit for bit
    (A2, B2, I2), g2 = run()
    assert np.array_equal(I1[:n], I2[:n]) and all(np.array_equal(x, y) for x, y in zip(g1, g2))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("rpt", [1, 4])
def test_tile_shape_matches_oracle(precision, rpt):
    """The ragged batch (degenerate crystals, a ragged last tile everywhere)
    at a fixed tile shape against the oracle, at the usual bounds."""
    from paper_2602_11709_amd.api import simulate
    b = ragged_batch()
    res = simulate(b, precision=precision, sf_rpt=rpt)
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, precision, f"ragged, {rpt} per lane")
    assert worst["ambiguous"] == 0
    print(precision, rpt, worst, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tile_shapes_agree_forward_and_adjoint(precision):
    """Structure factors, kept derivatives' gradients and the lattice rows of
    the adjoint at 1 and 4 reflections per lane against 2: crystals of 1 to
    700 atoms (single-wave and split items, fused atom pass and the
    atom-major path beyond 512 atoms), tails of every length."""
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = synth.random_triclinic(58, 40, atoms_lo=1, atoms_hi=700)
    grid = Grid(10.0, 0.02, 4001, 0.1, 8.0)
    dy = torch.randn(b.n_crystals, grid.n_points, dtype=torch.float64,
                     generator=torch.Generator().manual_seed(6)).cuda()
    out = {}
    for rpt in (2, 1, 4):
        xb = XrdBatch(b, precision=precision, keep_sf_derivs=True, grid_capacity=grid.n_points, sf_rpt=rpt)
        assert xb.sf_rpt == rpt
        refl = xb.enumerate()
        A, B, I = xb.structure_factors(refl)
        xb.pattern_forward(refl, I, grid)
        g = xb.pattern_backward(refl, grid, dy)
        torch.cuda.synchronize()
        n = int(xb.read_counts(refl)[0][-1])
        out[rpt] = ([t[:n].double().cpu().numpy() for t in (A, B)], [t.cpu().numpy() for t in g])
        del xb
    (A2, B2), g2 = out[2]
    scale = max(np.hypot(A2, B2).max(), 1e-300)
    tol_f = 1e-5 if precision == "mixed" else 1e-12
    tol_g = 1e-4 if precision == "mixed" else 1e-10
    for rpt in (1, 4):
        (A, B), g = out[rpt]
        assert np.max(np.abs(A - A2)) <= tol_f * scale and np.max(np.abs(B - B2)) <= tol_f * scale, rpt
        for name, a, c in zip(("dfrac", "dbfac", "dlat"), g2, g):
            err = np.max(np.abs(c - a)) / max(np.max(np.abs(a)), 1e-300)
            print(precision, rpt, name, f"{err:.2e}", flush=True)
            assert err <= tol_g, f"{rpt} {name}: {err:.3e}"
