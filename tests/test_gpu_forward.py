"""GPU forward pipeline (enumerate, structure factors, LP, sort, merge) against
the FP64 oracle, crystal by crystal and element by element."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.parity import compare_batch, compare_crystal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()  # fail loudly if the HIP library is missing


def run(batch, precision, **kw):
    from paper_2602_11709_amd.api import simulate
    return simulate(batch, precision=precision, **kw)


def ragged_batch():
    """Crystals spanning several enumeration/SF tiles with ragged tails, plus
    the degenerate cases: a crystal without atoms, one whose range holds no
    reflection, a single-atom crystal."""
    b = synth.random_triclinic(31, 12, atoms_lo=1, atoms_hi=120, len_lo=3.0, len_hi=13.0)
    parts = [b]
    coeff = b.sf_coeff
    empty_atoms = synth.CrystalBatch("t", np.array([[6.1, 7.2, 5.3, 80.0, 95.0, 101.0]]),
                                     np.array([0, 0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32),
                                     np.zeros(0), np.zeros(0), coeff, b.wavelength, np.array([10.0]),
                                     np.array([90.0]))
    no_refl = synth.CrystalBatch("t", np.array([[3.1, 3.2, 3.3, 90.0, 90.0, 90.0]]),
                                 np.array([0, 2], np.int64), np.random.default_rng(1).uniform(size=(2, 3)),
                                 np.array([1, 2], np.int32), np.ones(2), np.array([0.3, 0.9]), coeff,
                                 b.wavelength, np.array([10.0]), np.array([20.0]))
    # a crystal above the single-block sort limit (4096 reflections) between
    # small ones, so the bucket sort runs at a nonzero reflection offset
    big = synth.random_triclinic(33, 1, atoms_lo=30, atoms_hi=30, len_lo=13.5, len_hi=15.0)
    big.sf_coeff = coeff
    return concat([b.subset(range(6)), big, b.subset(range(6, 12)), empty_atoms, no_refl])


def concat(batches):
    lat = np.concatenate([x.lattice for x in batches])
    offs = [0]
    for x in batches:
        offs.extend((x.atom_offset[1:] + offs[-1]).tolist())
    return synth.CrystalBatch(
        "concat", lat, np.array(offs, np.int64), np.concatenate([x.frac for x in batches]),
        np.concatenate([x.species for x in batches]).astype(np.int32), np.concatenate([x.occ for x in batches]),
        np.concatenate([x.bfac for x in batches]), batches[0].sf_coeff, batches[0].wavelength,
        np.concatenate([x.two_theta_min for x in batches]), np.concatenate([x.two_theta_max for x in batches]),
        batches[0].merge_tol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rocksalt(precision):
    b = synth.rocksalt()
    res = run(b, precision)
    orc = oracle.pattern(b, 0)
    st = compare_crystal(res, 0, orc, precision, "rocksalt")
    assert st["n_refl"] == 586 and st["n_peaks"] == 23
    rs, ps = res.crystal(0)
    assert np.all(res.pk_mult[ps] % 2 == 0) and res.pk_mult[ps].sum() == 586
    print(precision, st, flush=True)


@pytest.mark.parametrize("precision,friedel", [("fp64", False), ("fp64", True), ("mixed", True),
                                               ("mixed", False)])
def test_ragged_batch(precision, friedel):
    b = ragged_batch()
    res = run(b, precision, friedel=friedel)
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, precision, "ragged")
    assert worst["ambiguous"] == 0
    rs, _ = res.crystal(b.n_crystals - 1)
    assert rs.stop == rs.start  # the crystal with no reflection in range
    big, _ = res.crystal(6)
    assert big.stop - big.start > 4096
    print(precision, friedel, worst, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triclinic_1024_full(precision):
    b = synth.triclinic_1024()
    res = run(b, precision)
    orcs = oracle.pattern_batch(b, threads=16)
    worst = compare_batch(res, b, orcs, precision, "triclinic_1024")
    assert worst["ambiguous"] == 0
    assert res.refl_offset[-1] == sum(o.n_refl for o in orcs)
    print(precision, "reflections", int(res.refl_offset[-1]), "peaks", int(res.peak_offset[-1]), worst, flush=True)


def test_fp64_and_mixed_runs_are_bitwise_deterministic():
    b = synth.random_triclinic(41, 64, atoms_hi=150)
    for precision in ("fp64", "mixed"):
        r1 = run(b, precision)
        r2 = run(b, precision)
        for f in ("hkl", "q", "two_theta", "A", "B", "I", "pk_two_theta", "pk_intensity", "pk_mult", "perm"):
            np.testing.assert_array_equal(getattr(r1, f), getattr(r2, f), err_msg=f"{precision} {f}")


def test_batch_equals_single_crystal_runs():
    b = synth.random_triclinic(43, 16, atoms_hi=80)
    whole = run(b, "fp64", friedel=False)
    for c in (0, 7, 15):
        one = run(b.subset([c]), "fp64", friedel=False)
        rs, ps = whole.crystal(c)
        np.testing.assert_array_equal(whole.I[rs], one.I)
        np.testing.assert_array_equal(whole.pk_intensity[ps], one.pk_intensity)


def test_threshold_drops_weak_peaks():
    b = synth.random_triclinic(47, 8, atoms_hi=60)
    res = run(b, "fp64", rel_threshold=0.05)
    for c in range(b.n_crystals):
        orc = oracle.pattern(b, c, threshold=0.05)
        rs, ps = res.crystal(c)
        assert ps.stop - ps.start == len(orc.pk_tt)
        np.testing.assert_array_equal(res.pk_mult[ps], orc.pk_mult)
        assert np.max(np.abs(res.pk_two_theta[ps] - orc.pk_tt), initial=0) <= 1e-9
        np.testing.assert_allclose(res.pk_intensity[ps], orc.pk_i, rtol=1e-10)
        np.testing.assert_allclose(res.pk_scaled[ps], orc.pk_y, rtol=1e-10)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_many_species_packs_atoms_in_their_own_launch(precision):
    """A species table of 300 rows (above what the enumeration launch carries
    for packing the atoms) takes the separate packing launch; crystals draw
    up to 40 species each, so their runs are short and many."""
    b = synth.random_triclinic(41, 10, atoms_lo=20, atoms_hi=90, species_per_crystal=40, pool=300)
    res = run(b, precision)
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, precision, "many species")
    assert worst["ambiguous"] == 0
    print(precision, worst, flush=True)


def test_offsets_formed_by_the_fill_for_mid_size_crystals():
    """Cells of 22-28 A (1.6e4-3.5e4 positive-half reflections: more than 64
    enumeration chunks of at most 256 candidates each, so a fill wavefront
    sums its crystal's chunk counts over several passes of its lanes, and
    below 256 chunks, so the fill forms the crystal offsets itself) between
    small crystals: every reflection list exactly, structure factors and
    strong peaks sampled, against the oracle."""
    from tests.parity import compare_crystal_sampled
    small = synth.random_triclinic(35, 6, atoms_lo=1, atoms_hi=30, len_lo=3.0, len_hi=9.0)
    mid = synth.random_triclinic(36, 4, atoms_lo=5, atoms_hi=20, len_lo=22.0, len_hi=28.0)
    mid.sf_coeff = small.sf_coeff
    b = concat([small.subset(range(3)), mid.subset([0, 1]), small.subset(range(3, 6)), mid.subset([2, 3])])
    res = run(b, "mixed")
    counts = np.diff(res.refl_offset) // 2
    print("positive-half reflections", counts.tolist(), flush=True)
    assert counts.max() > 64 * 256
    rng = np.random.default_rng(0)
    for c in range(b.n_crystals):
        compare_crystal_sampled(res, c, b, "mixed", rng, n_sample=200, n_strong=30, label="mid-size")


@pytest.mark.parametrize("case", ["2100 species", "1500-atom crystal"])
def test_separate_packing_launch_shapes(case):
    """The packing launch of its own in both shapes: 2100 species (eight
    wavefronts' cursor arrays would not fit in 64 KB of LDS, so one
    wavefront packs each crystal), and a 1500-atom crystal of 40 species
    between small ones (above 1024 atoms: eight wavefronts share the crystal,
    each a slice with many species runs, joined by one scan over (species,
    wavefront)).  Every reflection, structure factor and peak against the
    oracle."""
    if case == "2100 species":
        b = synth.random_triclinic(43, 6, atoms_lo=20, atoms_hi=90, species_per_crystal=40, pool=2100)
    else:
        small = synth.random_triclinic(44, 4, atoms_lo=5, atoms_hi=60, species_per_crystal=40, pool=300)
        big = synth.random_triclinic(45, 1, atoms_lo=1500, atoms_hi=1500, species_per_crystal=40, pool=300,
                                     len_lo=5.0, len_hi=7.0)
        big.sf_coeff = small.sf_coeff
        b = concat([small.subset([0, 1]), big, small.subset([2, 3])])
    res = run(b, "mixed")
    orcs = [oracle.pattern(b, c) for c in range(b.n_crystals)]
    worst = compare_batch(res, b, orcs, "mixed", case)
    assert worst["ambiguous"] == 0
    print(case, worst, flush=True)
