"""One launch over crystals of every size the batched path meets: the
degenerate cases (no atoms, no reflection in range), single-atom cells, cells
of the uneven 1024-crystal workload and two large cells of 2400-4700 atoms
with ~2e5 reflections each, interleaved so that heavy and light work share
every launch (heavy-first work tables, split-K items beside single-wavefront
ones, every sort size class in one merge).  Small crystals are checked
element by element against the oracle; the large ones exactly on their
reflection lists and peak partitions and on sampled structure factors and
strong peaks."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.parity import compare_crystal, compare_crystal_sampled
from tests.test_gpu_forward import ragged_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


def concat_species(batches):
    """Concatenate batches whose species tables differ: the tables are stacked
    and each batch's species indices shifted to its rows."""
    coeff = np.concatenate([x.sf_coeff for x in batches])
    shift = np.cumsum([0] + [x.n_species for x in batches[:-1]])
    offs = [0]
    for x in batches:
        offs.extend((x.atom_offset[1:] + offs[-1]).tolist())
    return synth.CrystalBatch(
        "mixed_sizes", np.concatenate([x.lattice for x in batches]), np.array(offs, np.int64),
        np.concatenate([x.frac for x in batches]),
        np.concatenate([x.species + s for x, s in zip(batches, shift)]).astype(np.int32),
        np.concatenate([x.occ for x in batches]), np.concatenate([x.bfac for x in batches]), coeff,
        batches[0].wavelength, np.concatenate([x.two_theta_min for x in batches]),
        np.concatenate([x.two_theta_max for x in batches]), batches[0].merge_tol)


def mixed_batch():
    t = synth.triclinic_1024()
    n = np.diff(t.atom_offset)
    rng = np.random.default_rng(5)
    ones = np.nonzero(n == 1)[0][:8]
    largest = np.argsort(n, kind="stable")[-6:]
    rest = rng.choice(np.setdiff1d(np.arange(t.n_crystals), np.concatenate([ones, largest])), 34, replace=False)
    pick = np.concatenate([ones[:4], largest[:3], rest[:17], ones[4:], largest[3:], rest[17:]])
    large = synth.large_cells()
    parts = [ragged_batch(), t.subset(pick[:24]), large.subset([9]), t.subset(pick[24:]), large.subset([1])]
    return concat_species(parts), parts


@pytest.mark.parametrize("precision,method", [("mixed", "direct"), ("fp64", "direct"), ("mixed", "auto"),
                                              ("fp64", "auto")])
def test_mixed_size_launch_against_oracle(precision, method):
    """With sf_method "auto" the two large cells take the row recurrence and
    the small ones the direct sum, in the same call (two concurrent launches),
    after the autotuner has chosen the threshold."""
    from paper_2602_11709_amd.api import simulate
    b, parts = mixed_batch()
    sizes = np.diff(b.atom_offset)
    big = [c for c in range(b.n_crystals) if sizes[c] >= 2000]
    assert len(big) == 2 and sizes.min() == 0 and 1 in sizes
    res = simulate(b, precision=precision, sf_method=method, autotune=method == "auto")
    small = [c for c in range(b.n_crystals) if c not in big]
    worst_small = {}
    for c in small:
        st = compare_crystal(res, c, oracle.pattern(b, c), precision, "mixed sizes", tol=b.merge_tol)
        for k, v in st.items():
            if isinstance(v, float):
                worst_small[k] = max(worst_small.get(k, 0.0), v)
    rng = np.random.default_rng(17)
    for c in big:
        st = compare_crystal_sampled(res, c, b, precision, rng, label="mixed sizes")
        print(precision, "large crystal", c, "atoms", int(sizes[c]), st, flush=True)
    print(precision, "small crystals", len(small), worst_small, "reflections", int(res.refl_offset[-1]), flush=True)


def test_first_structure_factor_call_captured_runs_on_one_stream():
    """Under sf_method "auto" this batch takes both the recurrence and the
    direct sum, which split over a side stream of the batch.  When the
    batch's first such call is captured in a graph there is no side stream yet
    (making one would end the capture), so the call runs on the batch's
    stream alone; its replays match a later eager (forked) call bit for bit."""
    from paper_2602_11709_amd.api import XrdBatch
    b, _ = mixed_batch()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xb = XrdBatch(b, precision="mixed", sf_method="auto")
        refl, sf = xb.new_reflections(), xb.new_sf()
        xb.enumerate(refl)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        xb.structure_factors(refl, sf)
    with torch.cuda.stream(s):
        xb.structure_factors(refl, sf)
    torch.cuda.synchronize()
    n = int(refl.refl_offset[-1])
    want = sf[2][:n].clone()
    print("reflections", n, flush=True)
    for rep in range(3):
        sf[2].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(sf[2][:n], want), f"replay {rep}"
