"""Gaussian-broadened pattern on the GPU against the oracle's broadening.

Two references: the oracle's whole pipeline (enumeration, structure factors,
broadening, all FP64) where it finishes in seconds, and the oracle's
broadening of the GPU's own reflection list and intensities, which isolates
the gather (entry lists, span ranges, windows) at any size, including
crystals sorted by the global-memory path."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.test_gpu_forward import ragged_batch

pytestmark = pytest.mark.gpu

# |y_gpu - y_ref| <= TOL * max|y_ref|.  Mixed gather: single-precision
# exponential of a double offset rounded to single (relative error of a term
# below 3e-7 within one sigma of its centre, ~4e-6 at the window edge where
# the Gaussian is e^-32), single-precision weights and sums of up to a few
# hundred terms (below 1e-6 relative); double everywhere in the plain path.
TOL = {"mixed": 1e-5, "fp64": 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


def gpu_pattern(batch, precision, grid, friedel=None):
    from paper_2602_11709_amd.api import XrdBatch
    xb = XrdBatch(batch, precision=precision, friedel=friedel, grid_capacity=grid.n_points)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    y = xb.pattern_forward(refl, I, grid)
    torch.cuda.synchronize()
    ro, _ = xb.read_counts(refl)
    n = int(ro[-1])
    return (y.cpu().numpy(), ro, refl.two_theta[:n].cpu().numpy(), I[:n].cpu().numpy())


def check_against_own_reflections(y, ro, tt, I, grid, precision, label):
    ga = (grid.t0, grid.dt, grid.n_points, grid.sigma, grid.window_sigmas)
    for c in range(len(ro) - 1):
        want = oracle.broaden(tt[ro[c]:ro[c + 1]], I[ro[c]:ro[c + 1]], *ga)
        scale = max(np.max(np.abs(want)), 1e-300)
        err = np.max(np.abs(y[c] - want)) / scale
        assert err <= TOL[precision], f"{label} crystal {c}: {err:.3e}"
        if not want.any():
            assert not y[c].any(), f"{label} crystal {c}: nonzero pattern without reflections"


@pytest.mark.parametrize("precision,friedel", [("mixed", True), ("fp64", False), ("fp64", True), ("mixed", False)])
def test_ragged_batch_pattern(precision, friedel):
    """Crystals of 0 to ~6000 reflections, an atomless crystal and one with no
    reflection in range; the grid starts below and ends above the
    reflections of some crystals, so windows are cut at both ends."""
    from paper_2602_11709_amd.api import Grid
    b = ragged_batch()
    grid = Grid(12.0, 0.017, 4501, 0.09, 8.0)
    y, ro, tt, I = gpu_pattern(b, precision, grid, friedel)
    check_against_own_reflections(y, ro, tt, I, grid, precision, "ragged")
    # the full oracle pipeline on a few of the small crystals
    ga = (grid.t0, grid.dt, grid.n_points, grid.sigma, grid.window_sigmas)
    for c in (0, 3, 7, 13):
        want = oracle.broadened(b, c, *ga)
        err = np.max(np.abs(y[c] - want)) / max(np.max(np.abs(want)), 1e-300)
        assert err <= (2e-5 if precision == "mixed" else 1e-10), f"crystal {c}: {err:.3e}"


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_large_cell_pattern(precision):
    """One crystal of the large-cell workload (~2.5e5 reflections, sorted by
    the global-memory path) on a 5751-point grid over its whole range."""
    from paper_2602_11709_amd.api import Grid
    b = synth.large_cells().subset([0])
    grid = Grid(5.0, 0.02, 5751, 0.1, 8.0)
    y, ro, tt, I = gpu_pattern(b, precision, grid)
    print(precision, "large cell reflections", int(ro[-1]), flush=True)
    assert ro[-1] > 1e5
    check_against_own_reflections(y, ro, tt, I, grid, precision, "large")


def test_sparse_grid_and_isolated_reflections():
    """A coarse grid (dt larger than the window) where most reflections reach
    no grid point and spans hold few entries."""
    from paper_2602_11709_amd.api import Grid
    b = synth.random_triclinic(41, 6, atoms_hi=40)
    grid = Grid(10.05, 1.7, 47, 0.1, 8.0)
    y, ro, tt, I = gpu_pattern(b, "mixed", grid)
    check_against_own_reflections(y, ro, tt, I, grid, "mixed", "sparse")


def test_grid_capacity_is_enforced():
    from paper_2602_11709_amd import capi
    from paper_2602_11709_amd.api import Grid, XrdBatch
    b = synth.rocksalt()
    xb = XrdBatch(b, precision="mixed", grid_capacity=1000)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    with pytest.raises(capi.XrdError):
        xb.pattern_forward(refl, I, Grid(10.0, 0.01, 1001, 0.1, 8.0))
    y = xb.pattern_forward(refl, I, Grid(10.0, 0.08, 1000, 0.1, 8.0))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()


def test_long_grid_uses_the_span_table_path():
    """A 40001-point grid (more spans than one block keeps in LDS) takes the
    path with the span tables in the workspace."""
    from paper_2602_11709_amd.api import Grid
    b = ragged_batch()
    grid = Grid(10.0, 0.002, 40001, 0.02, 8.0)
    y, ro, tt, I = gpu_pattern(b, "mixed", grid)
    check_against_own_reflections(y, ro, tt, I, grid, "mixed", "long grid")
