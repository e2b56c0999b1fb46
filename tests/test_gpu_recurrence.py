"""Structure factors by the row recurrence (sf_method "recurrence") against
the FP64 oracle at the direct path's bounds (|dF| <= 1e-12 sum|w| double,
4.5e-6 sum|w| mixed): every reflection of the ragged batch (degenerate
crystals, rows cut by the inner range limit, Friedel pairing on and off),
the whole 1024-crystal workload, sampled reflections of large cells, and the
quantities built on them (peaks, the kept derivatives that feed the
adjoint, graph replay, autotuning)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.parity import compare_batch, compare_crystal_sampled
from tests.test_gpu_forward import ragged_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


def run(batch, precision, **kw):
    from paper_2602_11709_amd.api import simulate
    return simulate(batch, precision=precision, sf_method="recurrence", **kw)


@pytest.mark.parametrize("precision,friedel", [("fp64", False), ("fp64", True), ("mixed", True),
                                               ("mixed", False)])
def test_ragged_batch_recurrence(precision, friedel):
    b = ragged_batch()
    res = run(b, precision, friedel=friedel)
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, precision, "ragged recurrence")
    assert worst["ambiguous"] == 0
    print(precision, friedel, worst, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triclinic_1024_recurrence(precision):
    b = synth.triclinic_1024()
    res = run(b, precision)
    orcs = oracle.pattern_batch(b, threads=16)
    worst = compare_batch(res, b, orcs, precision, "triclinic_1024 recurrence")
    assert worst["ambiguous"] == 0
    print(precision, worst, flush=True)


def test_inner_limit_splits_rows():
    """A range starting at 40 degrees removes the middle of the rows through
    the origin's neighbourhood: their runs break in two, and each piece is
    segmented on its own."""
    b = synth.random_triclinic(91, 6, atoms_lo=5, atoms_hi=40, len_lo=8.0, len_hi=12.0, tmin=40.0, tmax=100.0)
    for precision in ("fp64", "mixed"):
        res = run(b, precision, friedel=precision == "mixed")
        orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
        compare_batch(res, b, orcs, precision, "inner limit")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_large_cell_recurrence_sampled(precision):
    b = synth.large_cells().subset([3])
    res = run(b, precision)
    st = compare_crystal_sampled(res, 0, b, precision, np.random.default_rng(4), label="large recurrence")
    print(precision, st, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_recurrence_matches_direct_and_feeds_the_adjoint(precision):
    """Same reflections and peaks as the direct sum, structure factors within
    the precision's bound of each other, and the derivatives the recurrence
    forward keeps give the adjoint's gradients within the bar (1e-12 double,
    1e-4 mixed) of those from the direct forward."""
    from paper_2602_11709_amd.api import Grid, XrdBatch
    p = synth.gradient_problem(seed=12, n_crystals=6, atoms_lo=20, atoms_hi=300, grid_n=2001)
    grid = Grid(p.grid_t0, p.grid_dt, p.grid_n, p.sigma, p.window_sigmas)
    dy = torch.randn(p.batch.n_crystals, p.grid_n, generator=torch.Generator().manual_seed(2),
                     dtype=torch.float64).cuda()
    outs = {}
    for method in ("direct", "recurrence"):
        xb = XrdBatch(p.batch, precision=precision, grid_capacity=p.grid_n, keep_sf_derivs=True, sf_method=method)
        refl = xb.enumerate()
        A, B, I = xb.structure_factors(refl)
        y = xb.pattern_forward(refl, I, grid)
        g = xb.pattern_backward(refl, grid, dy)
        torch.cuda.synchronize()
        n = int(refl.refl_offset[-1])
        outs[method] = [t[:n].double().cpu().numpy() for t in (A, B, I)] + [y.cpu().numpy()] + \
            [t.cpu().numpy() for t in g]
    d, r = outs["direct"], outs["recurrence"]
    # both are within the bound of the oracle, so within twice it of each other
    absw = np.concatenate([oracle.pattern(p.batch, c).absw for c in range(p.batch.n_crystals)])
    assert len(absw) == len(d[0])
    bar_f = 2e-12 if precision == "fp64" else 9e-6
    rel = np.max(np.maximum(np.abs(r[0] - d[0]), np.abs(r[1] - d[1])) / absw)
    print(precision, "max |F_rec - F_direct| / sum|w|", rel, flush=True)
    assert rel <= bar_f
    bar = 1e-12 if precision == "fp64" else 1e-4
    for name, a, bb in zip(("dfrac", "dbfac", "dlattice"), d[4:], r[4:]):
        e = np.linalg.norm(a - bb) / np.linalg.norm(a)
        print(precision, name, "recurrence vs direct gradients rel", e, flush=True)
        assert e <= bar


def test_recurrence_graph_replay_and_autotune():
    """The recurrence step captured in a graph reproduces the eager result
    bit for bit over several replays; the autotuner picks a split for the
    recurrence's own table and the tuned results agree with the oracle."""
    from paper_2602_11709_amd.api import XrdBatch
    b = synth.random_triclinic(63, 40, atoms_hi=150)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xb = XrdBatch(b, precision="mixed", sf_method="recurrence")
        refl, sf, pk = xb.new_reflections(), xb.new_sf(), xb.new_peaks()
        xb.enumerate(refl)
        split = xb.autotune(refl)

    def step():
        xb.enumerate(refl)
        xb.structure_factors(refl, sf)
        xb.merge(refl, sf[2], pk)

    with torch.cuda.stream(s):
        step()
    torch.cuda.synchronize()
    n, m = int(refl.refl_offset[-1]), int(pk.peak_offset[-1])
    eager = [sf[2][:n].clone(), pk.intensity[:m].clone(), pk.mult[:m].clone()]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    for rep in range(3):
        sf[2].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [sf[2][:n], pk.intensity[:m], pk.mult[:m]]
        for a, bb in zip(eager, got):
            assert torch.equal(a, bb), f"replay {rep}"
    # tuned recurrence results against the oracle
    ro, po = xb.read_counts(refl, pk)
    inten = sf[2][:n].cpu().numpy()
    for c in (0, 17, 39):
        o = oracle.pattern(b, c)
        r0, r1 = int(ro[c]), int(ro[c + 1])
        lp = o.lp
        fabs = np.sqrt(o.fr ** 2 + o.fi ** 2)
        dF = 4.5e-6 * o.absw
        bound = lp * (2 * fabs * dF + dF * dF) + 1e-12 * o.inten
        assert np.all(np.abs(inten[r0:r1] - o.inten) <= bound)
    print("autotuned split", split, flush=True)
