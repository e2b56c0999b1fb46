"""Forward patterns of a crystal database streamed through one GPU in chunks.

The paper runs its calculator over whole structure databases (Section 4:
tens of thousands of MC3D and hundreds of thousands of COD structures, Mo
K-alpha, 2theta 2-60 degrees).  ``DatabaseStream`` does that on one GPU: the
crystals are cut into chunks of consecutive crystals; host threads plan the
coming chunks (``xrd_batch_create`` runs in C without the interpreter lock)
while the GPU computes the current one; each chunk's tables go to its
workspace on a copy stream, then enumeration, structure factors and the
merge run on the compute stream.  Two sets of device buffers alternate, so
chunk k + 1 is uploaded and enqueued while chunk k computes, and chunk k's
peaks are handed to the consumer (on the device, or copied to host memory)
while chunk k + 1 computes.

Every computation runs in the library's kernels; this module only plans,
allocates and orders the calls.
"""

from __future__ import annotations

import dataclasses
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Optional

import numpy as np
import torch

from . import capi
from .api import PRECISIONS, SF_METHODS
from .synth import CrystalBatch


@dataclasses.dataclass
class ChunkPeaks:
    """Peaks of one chunk (crystals first .. first + n_crystals - 1 of the
    database): CSR over the chunk's crystals.  Device tensors are views of
    the stream's buffers, valid only during the consumer call."""

    first: int
    n_crystals: int
    refl_offset: np.ndarray  # [n + 1] host
    peak_offset: np.ndarray  # [n + 1] host
    two_theta: torch.Tensor
    intensity: torch.Tensor
    scaled: torch.Tensor
    mult: torch.Tensor


class _Buffers:
    """Device buffers of one chunk in flight, grown on demand (with headroom)."""

    def __init__(self, device, precision):
        self.device = device
        self.precision = precision
        self.refl_cap = -1
        self.ws_bytes = -1
        self.n_c = -1
        self.done = None
        self.handle = None

    def ensure(self, refl_cap, ws_bytes, n_c):
        dev = self.device
        if refl_cap > self.refl_cap:
            cap = max(int(refl_cap * 1.25), 1)
            e = lambda dt: torch.empty(cap, dtype=dt, device=dev)
            self.h, self.k, self.l = e(torch.int16), e(torch.int16), e(torch.int16)
            self.q, self.tt, self.lp = e(torch.float64), e(torch.float64), e(torch.float64)
            sdt = torch.float32 if self.precision == "mixed" else torch.float64
            self.A, self.B, self.I = e(sdt), e(sdt), e(torch.float64)
            self.p_tt, self.p_i, self.p_y = e(torch.float64), e(torch.float64), e(torch.float64)
            self.p_mult, self.p_first, self.perm = e(torch.int32), e(torch.int64), e(torch.int64)
            self.refl_cap = cap
        if n_c > self.n_c:
            n = max(int(n_c * 1.25), 1) + 1
            self.refl_offset = torch.empty(n, dtype=torch.int64, device=dev)
            self.peak_offset = torch.empty(n, dtype=torch.int64, device=dev)
            self.n_c = n - 1
        if ws_bytes > self.ws_bytes:
            nb = int(ws_bytes * 1.25) + 256
            self.ws_raw = torch.empty(nb, dtype=torch.uint8, device=dev)
            self.ws = self.ws_raw.data_ptr() + (-self.ws_raw.data_ptr()) % 256
            self.ws_bytes = nb - 256

    def refl(self):
        return capi.xrd_refl(*(t.data_ptr() for t in (self.h, self.k, self.l, self.q, self.tt, self.lp,
                                                      self.refl_offset)))

    def peaks(self):
        return capi.xrd_peaks(*(t.data_ptr() for t in (self.p_tt, self.p_i, self.p_y, self.p_mult, self.p_first,
                                                       self.perm, self.peak_offset)))


class DatabaseStream:
    """Peaks (2theta, intensity, 0-100 scaled intensity, multiplicity) of every
    crystal of ``batch``, in chunks of ``chunk`` consecutive crystals.

    ``planners`` host threads plan chunks ahead of the GPU.  With ``ramp``
    the first chunks grow (an eighth, a quarter and a half of ``chunk``), so
    that the GPU starts after planning a small chunk rather than a full one.
    ``run`` calls
    ``consume(ChunkPeaks)`` once per chunk, in order, with device views of the
    chunk's peaks (and, with ``to_host``, host copies instead)."""

    def __init__(self, batch: CrystalBatch, chunk: int = 4096, precision: str = "mixed",
                 sf_method: str = "direct", planners: int = 4, device="cuda", ramp: bool = True):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        if sf_method not in SF_METHODS:
            raise ValueError(f"sf_method must be one of {list(SF_METHODS)}")
        if chunk < 1 or planners < 1:
            raise ValueError("chunk and planners must be >= 1")
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("DatabaseStream needs a GPU device; there is no CPU path")
        capi.lib()
        self.batch = batch
        self.precision = precision
        self.sf_method = sf_method
        self.planners = planners
        n = batch.n_crystals
        self.bounds = []
        c0, size = 0, max(1, chunk // 8) if ramp else chunk
        while c0 < n:
            self.bounds.append((c0, min(c0 + size, n)))
            c0 += size
            size = min(2 * size, chunk)
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        # every atom on the device once; a chunk's descriptor points into these
        self.frac = torch.as_tensor(batch.frac, **f64).contiguous()
        self.species = torch.as_tensor(batch.species, dtype=torch.int32, device=dev).contiguous()
        self.occ = torch.as_tensor(batch.occ, **f64).contiguous()
        self.bfac = torch.as_tensor(batch.bfac, **f64).contiguous()
        self.coeff = torch.as_tensor(batch.sf_coeff, **f64).contiguous()
        self.compute = torch.cuda.Stream(device=dev)
        self.copy = torch.cuda.Stream(device=dev)
        self.sets = [_Buffers(dev, precision), _Buffers(dev, precision)]
        self.stats = {}

    def _plan(self, k):
        """Plan chunk k on the host (any thread): (handle, sizes, kept arrays)."""
        b = self.batch
        c0, c1 = self.bounds[k]
        a0 = int(b.atom_offset[c0])
        keep = [np.ascontiguousarray(b.lattice[c0:c1]), np.ascontiguousarray(b.atom_offset[c0:c1 + 1] - a0),
                np.ascontiguousarray(b.two_theta_min[c0:c1]), np.ascontiguousarray(b.two_theta_max[c0:c1])]
        d = capi.xrd_batch_desc()
        d.n_crystals = c1 - c0
        d.n_species = b.n_species
        d.precision = PRECISIONS[self.precision]
        d.lattice, d.atom_offset, d.two_theta_min, d.two_theta_max = (a.ctypes.data for a in keep)
        d.wavelength = b.wavelength
        d.merge_tol = b.merge_tol
        d.rel_threshold = 0.0
        d.friedel = 1 if self.precision == "mixed" else 0
        d.sf_method = SF_METHODS[self.sf_method]
        d.forward_only = 1
        has_atoms = int(b.atom_offset[c1]) > a0
        d.frac = self.frac.data_ptr() + 24 * a0 if has_atoms else None
        d.species = self.species.data_ptr() + 4 * a0 if has_atoms else None
        d.occ = self.occ.data_ptr() + 8 * a0 if has_atoms else None
        d.bfac = self.bfac.data_ptr() + 8 * a0 if has_atoms else None
        d.sf_coeff = self.coeff.data_ptr()
        d.stream = self.copy.cuda_stream
        t0 = time.perf_counter()
        h = capi.xrd_batch_create(d)
        plan_s = time.perf_counter() - t0
        return h, capi.xrd_batch_sizes(h), keep, plan_s

    def run(self, consume: Optional[Callable[[ChunkPeaks], None]] = None, to_host: bool = False):
        """Process every chunk; returns timing statistics.  The wall time
        covers planning, uploads, the GPU work and the hand-over of every
        chunk's peaks."""
        n_chunks = len(self.bounds)
        stats = {"chunks": n_chunks, "plan_s": 0.0, "device_ms": 0.0, "reflections": 0, "peaks": 0}
        pool = ThreadPoolExecutor(max_workers=self.planners)
        futures = {}
        ahead = self.planners + 1

        def submit(k):
            if k < n_chunks and k not in futures:
                futures[k] = pool.submit(self._plan, k)

        events = []
        pending = None  # (k, set, start event, end event)
        t_start = time.perf_counter()
        try:
            for k in range(min(ahead, n_chunks)):
                submit(k)
            for k in range(n_chunks):
                h, sizes, keep, plan_s = futures.pop(k).result()
                submit(k + ahead)
                stats["plan_s"] += plan_s
                bufs = self.sets[k % 2]
                # the set's previous chunk (k - 2) has completed and been handed over
                if bufs.handle is not None:
                    capi.xrd_batch_destroy(bufs.handle)
                    bufs.handle = None
                bufs.ensure(int(sizes.refl_capacity), int(sizes.workspace_bytes), self.bounds[k][1] - self.bounds[k][0])
                # tables on the copy stream (the call waits for that copy only)
                capi.xrd_batch_upload(h, bufs.ws)
                capi.xrd_batch_set_stream(h, self.compute.cuda_stream)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(self.compute)
                refl, peaks = bufs.refl(), bufs.peaks()
                capi.xrd_enumerate_hkl(h, bufs.ws, refl)
                capi.xrd_structure_factors(h, bufs.ws, refl, bufs.A.data_ptr(), bufs.B.data_ptr(), bufs.I.data_ptr())
                capi.xrd_merge_peaks(h, bufs.ws, refl, bufs.I.data_ptr(), peaks)
                ev1.record(self.compute)
                bufs.handle = h
                bufs.keep = keep
                if pending is not None:
                    self._hand_over(pending, consume, to_host, stats, events)
                pending = (k, bufs, ev0, ev1)
            if pending is not None:
                self._hand_over(pending, consume, to_host, stats, events)
        finally:
            pool.shutdown(wait=True)
            for f in futures.values():
                hh = f.result()[0]
                capi.xrd_batch_destroy(hh)
        torch.cuda.synchronize(self.device)
        stats["wall_s"] = time.perf_counter() - t_start
        for bufs in self.sets:
            if bufs.handle is not None:
                capi.xrd_batch_destroy(bufs.handle)
                bufs.handle = None
        stats["device_ms"] = float(sum(a.elapsed_time(b) for a, b in events))
        stats["crystals"] = self.batch.n_crystals
        stats["patterns_per_s"] = self.batch.n_crystals / stats["wall_s"]
        stats["patterns_per_s_device"] = self.batch.n_crystals / max(stats["device_ms"] * 1e-3, 1e-12)
        self.stats = stats
        return stats

    def _hand_over(self, pending, consume, to_host, stats, events):
        k, bufs, ev0, ev1 = pending
        ev1.synchronize()
        events.append((ev0, ev1))
        c0, c1 = self.bounds[k]
        n = c1 - c0
        ro = bufs.refl_offset[: n + 1].cpu().numpy()
        po = bufs.peak_offset[: n + 1].cpu().numpy()
        m = int(po[-1])
        stats["reflections"] += int(ro[-1])
        stats["peaks"] += m
        if consume is None:
            return
        views = (bufs.p_tt[:m], bufs.p_i[:m], bufs.p_y[:m], bufs.p_mult[:m])
        if to_host:
            views = tuple(v.cpu() for v in views)
        consume(ChunkPeaks(c0, n, ro, po, *views))
