"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/xrd.h declares, and validates and plans batches on the host
(xrd_batch_create makes no HIP call)."""

import ctypes as C
import math
import re

import numpy as np
import pytest

import oracle
from paper_2602_11709_amd import capi, synth


def declared_functions():
    text = open(capi.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xrd_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 12
    lib = C.CDLL(capi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.SIGNATURES)
    assert capi.xrd_version().startswith("xrd-gfx950")


def make_desc(b: synth.CrystalBatch, keep, **over):
    """Descriptor with fake (never dereferenced) device pointers."""
    lat = np.ascontiguousarray(b.lattice)
    off = np.ascontiguousarray(b.atom_offset, np.int64)
    tmin = np.ascontiguousarray(b.two_theta_min)
    tmax = np.ascontiguousarray(b.two_theta_max)
    keep.extend([lat, off, tmin, tmax])
    d = capi.xrd_batch_desc()
    d.n_crystals = b.n_crystals
    d.n_species = b.n_species
    d.precision = capi.XRD_MIXED
    d.lattice, d.atom_offset = lat.ctypes.data, off.ctypes.data
    d.two_theta_min, d.two_theta_max = tmin.ctypes.data, tmax.ctypes.data
    d.wavelength, d.merge_tol, d.rel_threshold = b.wavelength, b.merge_tol, 0.0
    d.friedel = 1
    fake = 0x10000
    d.frac = d.species = d.occ = d.bfac = d.sf_coeff = fake
    d.stream = None
    for k, v in over.items():
        setattr(d, k, v)
    return d


def test_plan_capacity_bounds_oracle_counts():
    b = synth.random_triclinic(21, 40, atoms_hi=30)
    keep = []
    h = capi.xrd_batch_create(make_desc(b, keep))
    try:
        s = capi.xrd_batch_sizes(h)
        counts = [len(oracle.enumerate_hkl(b.lattice[c], b.wavelength, b.two_theta_min[c],
                                           b.two_theta_max[c])[2]) for c in range(b.n_crystals)]
        assert s.refl_capacity >= sum(counts)
        assert s.refl_capacity <= 6 * sum(counts)  # box / sphere volume ratio is modest
        assert s.n_atoms == b.n_atoms and s.n_crystals == 40
        assert s.workspace_bytes % 256 == 0 and s.workspace_bytes > 0
        assert s.half_capacity * 2 == s.refl_capacity
    finally:
        capi.xrd_batch_destroy(h)


def test_plan_capacity_per_crystal_tight_box():
    # one crystal at a time: capacity = (2H+1)(2K+1)(2L+1) - 1 with H = floor(gmax a)
    for lat in ([5.64, 5.64, 5.64, 90, 90, 90], [7.1, 3.3, 12.0, 64.0, 101.0, 117.0]):
        b = synth.rocksalt()
        b.lattice = np.array([lat], float)
        keep = []
        h = capi.xrd_batch_create(make_desc(b, keep))
        s = capi.xrd_batch_sizes(h)
        capi.xrd_batch_destroy(h)
        gmax = 2 * math.sin(math.radians(45.0)) / b.wavelength
        H, K, L = (math.floor(gmax * x) for x in lat[:3])
        assert s.refl_capacity == (2 * H + 1) * (2 * K + 1) * (2 * L + 1) - 1
        n = len(oracle.enumerate_hkl(lat, b.wavelength, 0.0, 90.0)[2])
        assert s.refl_capacity >= n


@pytest.mark.parametrize("field,value,code", [
    ("wavelength", 0.0, capi.XRD_ERR_INVALID_ARG),
    ("wavelength", -1.0, capi.XRD_ERR_INVALID_ARG),
    ("merge_tol", 0.0, capi.XRD_ERR_INVALID_ARG),
    ("rel_threshold", -0.1, capi.XRD_ERR_INVALID_ARG),
    ("precision", 7, capi.XRD_ERR_INVALID_ARG),
    ("friedel", 2, capi.XRD_ERR_INVALID_ARG),
    ("n_species", 0, capi.XRD_ERR_INVALID_ARG),
    ("n_crystals", -1, capi.XRD_ERR_INVALID_ARG),
    ("sf_coeff", None, capi.XRD_ERR_INVALID_ARG),
    ("frac", None, capi.XRD_ERR_INVALID_ARG),
    ("lattice", None, capi.XRD_ERR_INVALID_ARG),
])
def test_create_rejects_bad_arguments(field, value, code):
    b = synth.random_triclinic(3, 4, atoms_hi=10)
    keep = []
    d = make_desc(b, keep, **{field: value})
    h = C.c_void_p()
    rc = capi.lib().xrd_batch_create(C.byref(d), C.byref(h))
    assert rc == code
    assert not h.value
    assert capi.xrd_last_error()


def test_create_rejects_bad_cells_and_ranges():
    b = synth.random_triclinic(3, 3, atoms_hi=10)
    for lat, code in (([5, 5, 5, 120, 120, 120], capi.XRD_ERR_INVALID_CELL),
                      ([0, 5, 5, 90, 90, 90], capi.XRD_ERR_INVALID_CELL),
                      ([5, 5, 5, 90, 180, 90], capi.XRD_ERR_INVALID_CELL),
                      ([5e4, 5e4, 5e4, 90, 90, 90], capi.XRD_ERR_CAPACITY)):
        b2 = b.subset([0, 1, 2])
        b2.lattice[1] = lat
        keep = []
        with pytest.raises(capi.XrdError) as e:
            capi.xrd_batch_create(make_desc(b2, keep))
        assert e.value.code == code
    for lo, hi in ((-1.0, 90.0), (50.0, 40.0), (10.0, 180.0), (10.0, 10.0)):
        b2 = b.subset([0, 1, 2])
        b2.two_theta_min[2], b2.two_theta_max[2] = lo, hi
        keep = []
        with pytest.raises(capi.XrdError) as e:
            capi.xrd_batch_create(make_desc(b2, keep))
        assert e.value.code == capi.XRD_ERR_INVALID_ARG
        assert "crystal 2" in str(e.value)


def test_create_rejects_bad_offsets():
    b = synth.random_triclinic(3, 3, atoms_hi=10)
    b2 = b.subset([0, 1, 2])
    b2.atom_offset = b2.atom_offset.copy()
    b2.atom_offset[1] = b2.atom_offset[2] + 1
    keep = []
    with pytest.raises(capi.XrdError):
        capi.xrd_batch_create(make_desc(b2, keep))
    b3 = b.subset([0, 1, 2])
    b3.atom_offset = b3.atom_offset + 1
    with pytest.raises(capi.XrdError):
        capi.xrd_batch_create(make_desc(b3, keep))


def test_empty_batch_and_atomless_crystals_plan():
    b = synth.random_triclinic(3, 0)
    keep = []
    h = capi.xrd_batch_create(make_desc(b, keep, frac=None, species=None, occ=None, bfac=None))
    s = capi.xrd_batch_sizes(h)
    assert s.refl_capacity == 0 and s.n_crystals == 0
    capi.xrd_batch_destroy(h)
    capi.xrd_batch_destroy(None)


def test_device_calls_reject_null_workspace():
    b = synth.rocksalt()
    keep = []
    h = capi.xrd_batch_create(make_desc(b, keep))
    try:
        r = capi.xrd_refl()
        assert capi.lib().xrd_enumerate_hkl(h, None, C.byref(r)) == capi.XRD_ERR_INVALID_ARG
        assert capi.lib().xrd_enumerate_hkl(h, 0x1001, C.byref(r)) == capi.XRD_ERR_INVALID_ARG  # misaligned
        assert capi.lib().xrd_enumerate_hkl(h, 0x1000, C.byref(r)) == capi.XRD_ERR_INVALID_ARG  # null arrays
        g = capi.xrd_grid(10.0, 0.0, 100, 0.1, 8.0)
        assert capi.lib().xrd_pattern_forward(h, 0x1000, C.byref(r), None, C.byref(g), None) == \
            capi.XRD_ERR_INVALID_ARG
    finally:
        capi.xrd_batch_destroy(h)


def test_new_device_calls_validate_before_any_launch():
    """Families, Caglioti widths, texture and noise reject bad arguments on the
    host (every case fails validation before a kernel would be launched)."""
    b = synth.rocksalt()
    keep = []
    h = capi.xrd_batch_create(make_desc(b, keep))
    lib = capi.lib()
    fake = 0x1000  # never dereferenced: each call below fails validation first
    try:
        r = capi.xrd_refl(*([fake] * 7))
        p = capi.xrd_peaks(*([fake] * 7))
        pnull = capi.xrd_peaks(*([fake] * 5 + [None, fake]))  # perm missing
        ok = capi.XRD_ERR_INVALID_ARG
        assert lib.xrd_peak_families(h, fake, C.byref(r), C.byref(p), 7, fake, fake, fake, fake) == ok
        assert lib.xrd_peak_families(h, fake, C.byref(r), C.byref(pnull), 1, fake, fake, fake, fake) == ok
        assert lib.xrd_peak_families(h, fake, C.byref(r), C.byref(p), 1, fake, None, fake, fake) == ok
        assert lib.xrd_peak_families(h, fake, C.byref(r), None, 1, fake, fake, fake, fake) == ok
        g = capi.xrd_grid(10.0, 0.02, 100, 0.1, 8.0)
        assert lib.xrd_pattern_caglioti(h, fake, C.byref(r), fake, C.byref(g), float("nan"), 0.0, 0.01, 0.0, fake) == ok
        assert lib.xrd_pattern_caglioti(h, fake, C.byref(r), None, C.byref(g), 0.0, 0.0, 0.01, 0.0, fake) == ok
        assert lib.xrd_pattern_caglioti(h, fake, C.byref(r), fake, C.byref(g), 0.0, 0.0, 0.01, 1.5, fake) == ok
        bad = capi.xrd_grid(10.0, 0.0, 100, 0.1, 8.0)  # dt = 0
        assert lib.xrd_pattern_caglioti(h, fake, C.byref(r), fake, C.byref(bad), 0.0, 0.0, 0.01, 0.0, fake) == ok
        assert lib.xrd_preferred_orientation(h, fake, C.byref(r), None, fake, fake) == ok
        assert "non-NULL" in lib.xrd_last_error().decode() or lib.xrd_last_error()
    finally:
        capi.xrd_batch_destroy(h)


def test_noalloc_merge_scratch_size_and_rejection():
    """The allocation-free merge's scratch need is reported per batch, is part
    of the workspace's size, and a batch above the fixed scratch is refused
    before any HIP call (so this runs without a GPU)."""
    keep = []
    small = synth.random_triclinic(22, 20, atoms_hi=30)
    h = capi.xrd_batch_create(make_desc(small, keep))
    try:
        s = capi.xrd_batch_sizes(h)
        assert 0 < s.noalloc_merge_bytes < s.workspace_bytes
        assert s.noalloc_merge_bytes <= capi.XRD_NOALLOC_SCRATCH_BYTES
        assert s.noalloc_merge_bytes % 256 == 0
    finally:
        capi.xrd_batch_destroy(h)
    big = synth.random_triclinic(75, 1, atoms_lo=2, atoms_hi=2, len_lo=60.0, len_hi=62.0)
    h = capi.xrd_batch_create(make_desc(big, keep))
    try:
        s = capi.xrd_batch_sizes(h)
        assert s.noalloc_merge_bytes > capi.XRD_NOALLOC_SCRATCH_BYTES
        fake = 0x10000
        refl = capi.xrd_refl(*([fake] * 7))
        peaks = capi.xrd_peaks(*([fake] * 7))
        rc = capi.lib().xrd_merge_peaks_noalloc(h, C.byref(refl), fake, C.byref(peaks))
        assert rc == capi.XRD_ERR_CAPACITY
        assert "scratch" in capi.xrd_last_error()
        rc = capi.lib().xrd_merge_peaks_noalloc(h, C.byref(refl), None, C.byref(peaks))
        assert rc == capi.XRD_ERR_INVALID_ARG
    finally:
        capi.xrd_batch_destroy(h)


def test_sf_method_is_validated_and_sizes_the_workspace():
    keep = []
    b = synth.random_triclinic(23, 12, atoms_hi=40)
    h = capi.xrd_batch_create(make_desc(b, keep))
    direct = capi.xrd_batch_sizes(h).workspace_bytes
    capi.xrd_batch_destroy(h)
    h = capi.xrd_batch_create(make_desc(b, keep, sf_method=capi.XRD_SF_RECURRENCE))
    rec = capi.xrd_batch_sizes(h)
    capi.xrd_batch_destroy(h)
    # segment counts, their scan and starts: at most one segment per evaluated reflection
    assert rec.workspace_bytes >= direct + 16 * rec.half_capacity
    with pytest.raises(capi.XrdError) as ei:
        capi.xrd_batch_create(make_desc(b, keep, sf_method=3))
    assert ei.value.code == capi.XRD_ERR_INVALID_ARG


def test_tile_shape_is_validated_and_reported():
    """sf_rpt: 0 selects 2 reflections per lane, 1/2/4 are kept as given,
    anything else is refused; the workspace does not depend on it (it is
    sized for the finest shape)."""
    keep = []
    b = synth.random_triclinic(25, 9, atoms_hi=60)
    sizes = {}
    for rpt, expect in ((0, 2), (1, 1), (2, 2), (4, 4)):
        h = capi.xrd_batch_create(make_desc(b, keep, sf_rpt=rpt))
        try:
            assert capi.xrd_batch_get_sf_rpt(h) == expect
            sizes[rpt] = capi.xrd_batch_sizes(h).workspace_bytes
        finally:
            capi.xrd_batch_destroy(h)
    assert len(set(sizes.values())) == 1, sizes
    for bad in (3, 8, -1):
        with pytest.raises(capi.XrdError) as ei:
            capi.xrd_batch_create(make_desc(b, keep, sf_rpt=bad))
        assert ei.value.code == capi.XRD_ERR_INVALID_ARG


def test_combine_lines_rejects_bad_arguments():
    """Missing arrays or a negative weight are refused before any launch."""
    out = capi.xrd_line_peaks()
    with pytest.raises(capi.XrdError) as ei:
        capi.xrd_combine_lines(1, capi.xrd_line(), None, out, 0)
    assert ei.value.code == capi.XRD_ERR_INVALID_ARG
    with pytest.raises(capi.XrdError) as ei:
        capi.xrd_combine_lines(-1, capi.xrd_line(), None, out, 0)
    assert ei.value.code == capi.XRD_ERR_INVALID_ARG


def test_set_lattice_validates_before_any_device_work():
    """A cell needing a larger search box, or an invalid cell, is refused
    before anything is copied (host only)."""
    keep = []
    b = synth.random_triclinic(24, 3, atoms_hi=10)
    h = capi.xrd_batch_create(make_desc(b, keep))
    try:
        fake_ws = 0x100000  # 256-aligned, never touched on these paths
        bigger = np.ascontiguousarray(b.lattice.copy())
        bigger[1, 0] *= 1.5
        assert capi.xrd_batch_set_lattice(h, bigger.ctypes.data, fake_ws) == capi.XRD_ERR_CAPACITY
        assert "larger search box" in capi.xrd_last_error()
        flat = np.ascontiguousarray(b.lattice.copy())
        flat[0, 3:] = 120.0
        with pytest.raises(capi.XrdError) as ei:
            capi.xrd_batch_set_lattice(h, flat.ctypes.data, fake_ws)
        assert ei.value.code == capi.XRD_ERR_INVALID_CELL
    finally:
        capi.xrd_batch_destroy(h)
