"""The allocation-free merge (xrd_merge_peaks_noalloc, fixed device scratch)
against the workspace merge (xrd_merge_peaks) on the same reflections and
intensities: every output bit for bit (both run the same sort and merge
kernels; the variant only moves their working storage and runs them on one
stream).  Two calls in a row, the second on a smaller batch of another
layout, so the second must not depend on what the first left in the shared
scratch."""

import numpy as np
import pytest
import torch

from paper_2602_11709_amd import capi, synth
from tests.test_gpu_forward import concat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    capi.lib()


def first_batch():
    """Crystals of every sort size class: tiny and small cells, two of the
    mid class (8192-16384 reflections) and one above the single-block limits
    (capacity ~1e5: sorted in global memory over many blocks, with its
    bucket tables in the fixed scratch too)."""
    small = synth.random_triclinic(71, 90, atoms_hi=80)
    big = synth.random_triclinic(72, 1, atoms_lo=20, atoms_hi=20, len_lo=24.0, len_hi=26.0)
    mid = synth.random_triclinic(73, 2, atoms_lo=10, atoms_hi=10, len_lo=13.0, len_hi=15.0)
    big.sf_coeff = mid.sf_coeff = small.sf_coeff
    return concat([small.subset(range(45)), big, mid, small.subset(range(45, 90))])


def merged(batch, precision, rel_threshold, noalloc):
    from paper_2602_11709_amd.api import XrdBatch
    xb = XrdBatch(batch, precision=precision, rel_threshold=rel_threshold)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    ref = xb.merge(refl, I)
    got = xb.new_peaks()
    for t in (got.two_theta, got.intensity, got.scaled):
        t.fill_(float("nan"))
    for t in (got.mult, got.first, got.perm, got.peak_offset):
        t.fill_(-7)
    assert xb.sizes.noalloc_merge_bytes <= capi.XRD_NOALLOC_SCRATCH_BYTES
    print("noalloc", batch.n_crystals, "crystals", precision, "scratch bytes", xb.sizes.noalloc_merge_bytes,
          flush=True)
    noalloc(xb, refl, I, got)
    torch.cuda.synchronize()
    return xb, refl, I, ref, got


def check_equal(refl, ref, got):
    ro = refl.refl_offset.cpu()
    po = ref.peak_offset.cpu()
    assert torch.equal(po, got.peak_offset.cpu())
    n, m = int(ro[-1]), int(po[-1])
    assert m > 0 and n > 0
    for name in ("two_theta", "intensity", "scaled", "mult", "first"):
        a, b = getattr(ref, name)[:m], getattr(got, name)[:m]
        assert torch.equal(a, b), name
    assert torch.equal(ref.perm[:n], got.perm[:n])


def test_noalloc_merge_matches_workspace_merge_twice():
    call = lambda xb, refl, I, p: capi.xrd_merge_peaks_noalloc(xb.handle, refl.c(), I.data_ptr(), p.c())
    b1 = first_batch()
    xb1, refl1, I1, ref1, got1 = merged(b1, "mixed", 0.0, call)
    check_equal(refl1, ref1, got1)
    # second call: a smaller batch, no Friedel pairing (another scratch
    # layout), a relative threshold; the scratch still holds the first call's data
    b2 = synth.random_triclinic(74, 30, atoms_hi=60)
    xb2, refl2, _, ref2, got2 = merged(b2, "fp64", 1e-3, call)
    assert xb2.sizes.noalloc_merge_bytes < xb1.sizes.noalloc_merge_bytes
    check_equal(refl2, ref2, got2)
    # and the first batch once more after the second
    got1b = xb1.new_peaks()
    call(xb1, refl1, I1, got1b)
    torch.cuda.synchronize()
    check_equal(refl1, ref1, got1b)


def test_noalloc_merge_rejects_oversized_batch():
    """A batch whose merge needs more than the fixed scratch is refused with
    XRD_ERR_CAPACITY before any work is enqueued."""
    from paper_2602_11709_amd.api import XrdBatch
    b = synth.random_triclinic(75, 1, atoms_lo=2, atoms_hi=2, len_lo=60.0, len_hi=62.0)
    xb = XrdBatch(b, precision="mixed")
    assert xb.sizes.noalloc_merge_bytes > capi.XRD_NOALLOC_SCRATCH_BYTES
    refl = xb.new_reflections()
    _, _, I = xb.new_sf()
    with pytest.raises(capi.XrdError) as ei:
        capi.xrd_merge_peaks_noalloc(xb.handle, refl.c(), I.data_ptr(), xb.new_peaks().c())
    assert ei.value.code == capi.XRD_ERR_CAPACITY
