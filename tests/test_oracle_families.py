"""Pins of the oracle's grouping of symmetry-equivalent reflections.

The lattice rule is pinned by the orders of the lattice point groups (the
seven holohedries) and by the textbook reflection multiplicities of their
Laue classes (International Tables for Crystallography, Vol. A), on peaks
built here as every (h, k, l) of a small box with the same 1/d^2 as a given
reflection.  The index rule is pinned by its definition on hand-made lists,
and by agreeing with the lattice rule on cubic and hexagonal lattices."""
import itertools

import numpy as np
import pytest

import oracle

CUBIC = [4.0, 4.0, 4.0, 90.0, 90.0, 90.0]
TETRA = [3.7, 3.7, 5.3, 90.0, 90.0, 90.0]
HEXA = [3.1, 3.1, 5.2, 90.0, 90.0, 120.0]
RHOMB = [4.1, 4.1, 4.1, 71.0, 71.0, 71.0]
ORTHO = [3.1, 4.3, 5.7, 90.0, 90.0, 90.0]
MONO = [3.1, 4.3, 5.7, 90.0, 101.0, 90.0]
TRIC = [3.1, 4.3, 5.7, 81.0, 97.0, 103.0]


def peak_of(lattice, rep, box=5):
    """Every (h, k, l) of the box with the same 1/d^2 as rep, in ascending
    (h, k, l) order: one peak of a powder pattern."""
    _, gs, _ = oracle.cell(lattice)
    q0 = oracle.q_of(gs, *rep)
    rng = range(-box, box + 1)
    return [t for t in itertools.product(rng, rng, rng) if abs(oracle.q_of(gs, *t) - q0) <= 1e-9 * q0]


def families(lattice, rule, members):
    fam, n_fam, label, mult = oracle.peak_families(lattice, rule, [0], [len(members)], members)
    nf = int(n_fam[0])
    return [(tuple(int(v) for v in label[f]), int(mult[f])) for f in range(nf)], fam


@pytest.mark.parametrize("lattice,order", [(CUBIC, 48), (HEXA, 24), (TETRA, 16), (RHOMB, 12), (ORTHO, 8),
                                           (MONO, 4), (TRIC, 2)])
def test_lattice_point_group_orders(lattice, order):
    ops = oracle.lattice_ops(lattice)
    assert len(ops) == order
    # a group: closed under products, contains the identity and -identity
    keys = {o.tobytes() for o in ops}
    assert np.eye(3, dtype=np.int32).tobytes() in keys and (-np.eye(3, dtype=np.int32)).tobytes() in keys
    for a in ops[:12]:
        for b in ops[:12]:
            assert (a @ b).astype(np.int32).tobytes() in keys


# (lattice, representative, multiplicity of its family in the lattice's Laue class)
LAUE = [
    (CUBIC, (1, 0, 0), 6), (CUBIC, (1, 1, 0), 12), (CUBIC, (1, 1, 1), 8), (CUBIC, (2, 1, 0), 24),
    (CUBIC, (2, 1, 1), 24), (CUBIC, (3, 2, 1), 48),
    (TETRA, (1, 0, 0), 4), (TETRA, (0, 0, 1), 2), (TETRA, (1, 1, 0), 4), (TETRA, (1, 0, 1), 8),
    (TETRA, (1, 1, 1), 8), (TETRA, (2, 1, 0), 8), (TETRA, (2, 1, 1), 16),
    (HEXA, (1, 0, 0), 6), (HEXA, (0, 0, 1), 2), (HEXA, (1, 1, 0), 6), (HEXA, (1, 0, 1), 12),
    (HEXA, (1, 1, 1), 12), (HEXA, (2, 1, 0), 12), (HEXA, (2, 1, 1), 24),
    (RHOMB, (1, 0, 0), 6), (RHOMB, (1, 1, 1), 2), (RHOMB, (1, 1, 0), 6), (RHOMB, (1, -1, 0), 6),
    (RHOMB, (2, 1, 0), 12),
    (ORTHO, (1, 0, 0), 2), (ORTHO, (1, 1, 0), 4), (ORTHO, (1, 1, 1), 8),
    (MONO, (1, 1, 1), 4), (MONO, (0, 1, 0), 2), (MONO, (1, 0, 1), 2), (MONO, (1, 1, 0), 4),
    (TRIC, (1, 1, 1), 2), (TRIC, (1, 0, 0), 2),
]


@pytest.mark.parametrize("lattice,rep,mult", LAUE)
def test_laue_multiplicities(lattice, rep, mult):
    members = peak_of(lattice, rep)
    assert len(members) == mult  # the peak is exactly one family (no accidental coincidence)
    fams, fam = families(lattice, oracle.FAM_LATTICE, members)
    assert fams == [(max(members), mult)]
    assert (fam == 0).all()


def test_accidental_coincidence_cubic():
    # h^2 + k^2 + l^2 = 9 and 25: two families share one powder line each
    fams, _ = families(CUBIC, oracle.FAM_LATTICE, peak_of(CUBIC, (3, 0, 0)))
    assert fams == [((3, 0, 0), 6), ((2, 2, 1), 24)]
    fams, _ = families(CUBIC, oracle.FAM_LATTICE, peak_of(CUBIC, (5, 0, 0), box=6))
    assert fams == [((5, 0, 0), 6), ((4, 3, 0), 24)]


def test_labels_are_largest_members():
    fams, _ = families(HEXA, oracle.FAM_LATTICE, peak_of(HEXA, (1, 1, 0)))
    assert fams == [((2, -1, 0), 6)]
    fams, _ = families(TETRA, oracle.FAM_LATTICE, peak_of(TETRA, (2, 1, 1)))
    assert fams == [((2, 1, 1), 16)]


@pytest.mark.parametrize("lattice,rep", [(CUBIC, (3, 2, 1)), (CUBIC, (3, 0, 0)), (HEXA, (2, 1, 1)),
                                         (HEXA, (1, 0, 0)), (HEXA, (1, 1, 0))])
def test_index_rule_matches_lattice_rule_on_cubic_and_hexagonal(lattice, rep):
    members = peak_of(lattice, rep)
    a = families(lattice, oracle.FAM_INDICES, members)
    b = families(lattice, oracle.FAM_LATTICE, members)
    assert a[0] == b[0] and (a[1] == b[1]).all()


def test_index_rule_definition():
    members = [(1, 2, 0), (2, 1, 0), (1, 0, 0), (0, -1, 2), (0, 0, -1)]
    fams, fam = families(ORTHO, oracle.FAM_INDICES, members)
    assert fams == [((2, 1, 0), 3), ((1, 0, 0), 2)]
    assert fam.tolist() == [0, 0, 1, 0, 1]
    # the lattice rule keeps them apart on this lattice (only sign changes of each index)
    fams, _ = families(ORTHO, oracle.FAM_LATTICE, members)
    assert [m for _, m in fams] == [1, 1, 1, 1, 1]
    # 4-index form on a hexagonal lattice only: (1, 0, 0) ~ (1, -1, 0)
    pair = [(1, 0, 0), (1, -1, 0)]
    assert families(HEXA, oracle.FAM_INDICES, pair)[0] == [((1, 0, 0), 2)]
    assert families(ORTHO, oracle.FAM_INDICES, pair)[0] == [((1, 0, 0), 1), ((1, -1, 0), 1)]


def test_hexagonal_detection():
    assert oracle.is_hexagonal(HEXA)
    assert not oracle.is_hexagonal([3.1, 3.1, 5.2, 90.0, 90.0, 60.0])
    assert not oracle.is_hexagonal([3.1, 3.2, 5.2, 90.0, 90.0, 120.0])
    assert not oracle.is_hexagonal(CUBIC)


def test_several_peaks_and_degenerate_cases():
    p1, p2 = peak_of(CUBIC, (1, 1, 1)), [(0, 0, 1)]
    fam, n_fam, label, mult = oracle.peak_families(CUBIC, oracle.FAM_LATTICE, [0, 8], [8, 1], p1 + p2)
    assert n_fam.tolist() == [1, 1]
    assert tuple(label[0]) == (1, 1, 1) and mult[0] == 8
    assert tuple(label[8]) == (0, 0, 1) and mult[8] == 1 and fam[8] == 0
    fam, n_fam, _, _ = oracle.peak_families(CUBIC, oracle.FAM_LATTICE, [], [], np.zeros((0, 3)))
    assert len(fam) == 0 and len(n_fam) == 0
    with pytest.raises(ValueError):
        oracle.peak_families([1, 1, 1, 90, 90, 200], oracle.FAM_LATTICE, [0], [1], [(1, 0, 0)])
    with pytest.raises(ValueError):
        oracle.peak_families(CUBIC, 7, [0], [1], [(1, 0, 0)])
