"""The database stream (chunks of consecutive crystals planned on host
threads while the GPU computes, two sets of buffers alternating) gives the
same peaks, bit for bit, as one batch of the same crystals, and those agree
with the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2602_11709_amd import synth
from tests.parity import compare_crystal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2602_11709_amd import capi
    capi.lib()


@pytest.mark.parametrize("precision,method", [("mixed", "direct"), ("fp64", "auto")])
def test_stream_matches_one_batch_and_oracle(precision, method):
    from paper_2602_11709_amd.api import simulate
    from paper_2602_11709_amd.stream import DatabaseStream
    b = synth.database_stream(n_crystals=2600)
    got = {}

    def consume(cp):
        got[cp.first] = cp

    st = DatabaseStream(b, chunk=600, precision=precision, sf_method=method, planners=3).run(consume, to_host=True)
    print(precision, method, {k: v for k, v in st.items() if not isinstance(v, float) or v < 1e9}, flush=True)
    # chunks of 75, 150, 300, then 600 (the last one ragged)
    assert sorted(got) == [0, 75, 225, 525, 1125, 1725, 2325]
    whole = simulate(b, precision=precision, sf_method=method)
    assert st["reflections"] == int(whole.refl_offset[-1]) and st["peaks"] == int(whole.peak_offset[-1])
    for c0, cp in got.items():
        np.testing.assert_array_equal(cp.refl_offset, whole.refl_offset[c0:c0 + cp.n_crystals + 1]
                                      - whole.refl_offset[c0])
        p0, p1 = int(whole.peak_offset[c0]), int(whole.peak_offset[c0 + cp.n_crystals])
        np.testing.assert_array_equal(cp.peak_offset, whole.peak_offset[c0:c0 + cp.n_crystals + 1] - p0)
        np.testing.assert_array_equal(cp.two_theta.numpy(), whole.pk_two_theta[p0:p1])
        np.testing.assert_array_equal(cp.intensity.numpy(), whole.pk_intensity[p0:p1])
        np.testing.assert_array_equal(cp.mult.numpy(), whole.pk_mult[p0:p1])
    # and the one batch against the oracle on a sample spanning every chunk
    rng = np.random.default_rng(8)
    for c in sorted(rng.choice(b.n_crystals, 40, replace=False)):
        compare_crystal(whole, int(c), oracle.pattern(b, int(c)), precision, "stream sample", tol=b.merge_tol)


def test_stream_device_hand_over_and_empty_chunks():
    """Peaks handed over as device views (valid during the call) match the
    host copies; crystals without atoms or reflections inside chunks are
    fine."""
    from paper_2602_11709_amd.stream import DatabaseStream
    from tests.test_gpu_forward import ragged_batch
    b = ragged_batch()
    dev = []
    DatabaseStream(b, chunk=5, planners=2, ramp=False).run(lambda cp: dev.append(cp.intensity.cpu().numpy().copy()))
    host = []
    DatabaseStream(b, chunk=5, planners=2, ramp=False).run(lambda cp: host.append(cp.intensity.numpy().copy()),
                                                           to_host=True)
    assert len(dev) == len(host) == 3
    for a, c in zip(dev, host):
        np.testing.assert_array_equal(a, c)


def test_peak_numbering_with_and_without_the_scan():
    """Batches of up to 4096 crystals number their peaks inside the move
    kernel, larger ones with a scan first: 5000 crystals as one batch (scan)
    and as two chunks of 2500 (in-kernel sums) give the same offsets and
    peaks bit for bit."""
    from paper_2602_11709_amd.api import simulate
    from paper_2602_11709_amd.stream import DatabaseStream
    b = synth.database_stream(n_crystals=5000)
    got = {}
    DatabaseStream(b, chunk=2500, precision="mixed", planners=2, ramp=False).run(
        lambda cp: got.__setitem__(cp.first, cp), to_host=True)
    whole = simulate(b, precision="mixed")
    assert sorted(got) == [0, 2500]
    for c0, cp in got.items():
        p0 = int(whole.peak_offset[c0])
        np.testing.assert_array_equal(cp.peak_offset, whole.peak_offset[c0:c0 + cp.n_crystals + 1] - p0)
        p1 = int(whole.peak_offset[c0 + cp.n_crystals])
        np.testing.assert_array_equal(cp.two_theta.numpy(), whole.pk_two_theta[p0:p1])
        np.testing.assert_array_equal(cp.intensity.numpy(), whole.pk_intensity[p0:p1])
        np.testing.assert_array_equal(cp.mult.numpy(), whole.pk_mult[p0:p1])
