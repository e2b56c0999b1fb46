"""PyTorch front end: device buffers and streams around the C ABI.

PyTorch supplies device memory and the stream; every computation runs in the
library's kernels.  ``XrdBatch`` owns one batch handle, its workspace and the
device copies of the atom arrays; its methods mirror the C calls.
``simulate`` runs the whole forward pipeline and returns host arrays, and
``XrdPattern`` is the differentiable broadened pattern (``torch.autograd``)
whose backward is the library's hand-written adjoint.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np
import torch

from . import capi
from .synth import CrystalBatch

PRECISIONS = {"fp64": capi.XRD_FP64, "mixed": capi.XRD_MIXED}
SF_METHODS = {"direct": capi.XRD_SF_DIRECT, "recurrence": capi.XRD_SF_RECURRENCE, "auto": capi.XRD_SF_AUTO}


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


@dataclasses.dataclass
class Grid:
    t0: float
    dt: float
    n_points: int
    sigma: float
    window_sigmas: float = 8.0

    def c(self) -> capi.xrd_grid:
        return capi.xrd_grid(self.t0, self.dt, int(self.n_points), self.sigma, self.window_sigmas)


@dataclasses.dataclass
class Reflections:
    h: torch.Tensor
    k: torch.Tensor
    l: torch.Tensor
    q: torch.Tensor
    two_theta: torch.Tensor
    lp: torch.Tensor
    refl_offset: torch.Tensor

    def c(self) -> capi.xrd_refl:
        return capi.xrd_refl(*(t.data_ptr() for t in (self.h, self.k, self.l, self.q, self.two_theta, self.lp,
                                                      self.refl_offset)))


@dataclasses.dataclass
class Peaks:
    two_theta: torch.Tensor
    intensity: torch.Tensor
    scaled: torch.Tensor
    mult: torch.Tensor
    first: torch.Tensor
    perm: torch.Tensor
    peak_offset: torch.Tensor

    def c(self) -> capi.xrd_peaks:
        return capi.xrd_peaks(*(t.data_ptr() for t in (self.two_theta, self.intensity, self.scaled, self.mult,
                                                       self.first, self.perm, self.peak_offset)))


class XrdBatch:
    """One planned batch on one GPU.

    Host inputs (lattice, atom offsets, 2theta ranges) are read at
    construction; atom arrays are copied to the device once and kept alive
    here.  All work goes to the stream that is current at construction.
    ``frac``/``bfac`` may be given as device tensors (float64) to override
    the batch's arrays (the differentiable path does this).
    ``grid_capacity`` bounds the grid of broadened-pattern calls (0: 16384
    points).  With ``keep_sf_derivs`` the structure-factor call also keeps
    dF/d(s^2) for a following ``pattern_backward`` on the same reflections,
    which then skips its own pass over the atoms.  ``sf_method`` picks how the
    structure factors sum over the atoms: "direct" (sin/cos of every term),
    "recurrence" (stepped along reciprocal-lattice rows from exact seeds) or
    "auto" (the recurrence for crystals with many atoms and long rows).
    ``forward_only`` leaves out the adjoint's tables and buffers (no
    ``pattern_backward`` on this batch).  ``sf_rpt`` fixes the tile shape of
    the direct sums (reflections per lane: 1, 2 or 4); 0 starts at 2 and lets
    ``autotune`` choose."""

    def __init__(self, batch: CrystalBatch, precision: str = "mixed", friedel: Optional[bool] = None,
                 rel_threshold: float = 0.0, device="cuda", frac: Optional[torch.Tensor] = None,
                 bfac: Optional[torch.Tensor] = None, lattice: Optional[np.ndarray] = None,
                 two_theta_range: Optional[tuple] = None, grid_capacity: int = 0,
                 keep_sf_derivs: bool = False, sf_method: str = "direct", forward_only: bool = False,
                 sf_rpt: int = 0):
        if sf_rpt not in (0, 1, 2, 4):
            raise ValueError("sf_rpt must be 0, 1, 2 or 4")
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        if sf_method not in SF_METHODS:
            raise ValueError(f"sf_method must be one of {list(SF_METHODS)}")
        self.sf_method = sf_method
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("XrdBatch needs a GPU device; there is no CPU path")
        self.precision = precision
        self.friedel = (precision == "mixed") if friedel is None else bool(friedel)
        self.batch = batch
        dev = self.device
        self.stream = torch.cuda.current_stream(dev)
        f64 = dict(dtype=torch.float64, device=dev)
        self.frac = (frac if frac is not None else torch.as_tensor(batch.frac, **f64)).contiguous()
        self.bfac = (bfac if bfac is not None else torch.as_tensor(batch.bfac, **f64)).contiguous()
        self.species = torch.as_tensor(batch.species, dtype=torch.int32, device=dev).contiguous()
        self.occ = torch.as_tensor(batch.occ, **f64).contiguous()
        self.coeff = torch.as_tensor(batch.sf_coeff, **f64).contiguous()
        self.lattice = np.ascontiguousarray(batch.lattice if lattice is None else lattice, dtype=np.float64)
        self.atom_offset = np.ascontiguousarray(batch.atom_offset, dtype=np.int64)
        if two_theta_range is None:
            self.tmin = np.ascontiguousarray(batch.two_theta_min, dtype=np.float64)
            self.tmax = np.ascontiguousarray(batch.two_theta_max, dtype=np.float64)
        else:
            self.tmin = np.full(batch.n_crystals, float(two_theta_range[0]))
            self.tmax = np.full(batch.n_crystals, float(two_theta_range[1]))
        d = capi.xrd_batch_desc()
        d.n_crystals = batch.n_crystals
        d.n_species = batch.n_species
        d.precision = PRECISIONS[precision]
        d.lattice = self.lattice.ctypes.data
        d.atom_offset = self.atom_offset.ctypes.data
        d.two_theta_min = self.tmin.ctypes.data
        d.two_theta_max = self.tmax.ctypes.data
        d.wavelength = batch.wavelength
        d.merge_tol = batch.merge_tol
        d.rel_threshold = rel_threshold
        d.friedel = 1 if self.friedel else 0
        d.grid_capacity = int(grid_capacity)
        d.keep_sf_derivs = 1 if keep_sf_derivs else 0
        d.sf_method = SF_METHODS[sf_method]
        d.forward_only = 1 if forward_only else 0
        d.sf_rpt = sf_rpt
        d.frac = _p(self.frac) if batch.n_atoms else None
        d.species = _p(self.species) if batch.n_atoms else None
        d.occ = _p(self.occ) if batch.n_atoms else None
        d.bfac = _p(self.bfac) if batch.n_atoms else None
        d.sf_coeff = _p(self.coeff)
        d.stream = self.stream.cuda_stream
        self.desc = d
        self.handle = None
        t_plan = time.perf_counter()
        self.handle = capi.xrd_batch_create(d)
        self.plan_ms = (time.perf_counter() - t_plan) * 1e3  # host planning alone
        self.sizes = capi.xrd_batch_sizes(self.handle)
        nb = int(self.sizes.workspace_bytes)
        self._ws_raw = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        self.ws = self._ws_raw.data_ptr() + (-self._ws_raw.data_ptr()) % 256
        capi.xrd_batch_upload(self.handle, self.ws)

    def __del__(self):
        h = getattr(self, "handle", None)
        destroy = getattr(capi, "xrd_batch_destroy", None)
        if h and callable(destroy):  # the module may already be torn down at interpreter exit
            try:
                destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def n_crystals(self):
        return self.batch.n_crystals

    @property
    def refl_capacity(self):
        return int(self.sizes.refl_capacity)

    # ---- allocation --------------------------------------------------------

    def new_reflections(self) -> Reflections:
        n = max(self.refl_capacity, 1)
        dev = self.device
        return Reflections(
            h=torch.empty(n, dtype=torch.int16, device=dev), k=torch.empty(n, dtype=torch.int16, device=dev),
            l=torch.empty(n, dtype=torch.int16, device=dev), q=torch.empty(n, dtype=torch.float64, device=dev),
            two_theta=torch.empty(n, dtype=torch.float64, device=dev),
            lp=torch.empty(n, dtype=torch.float64, device=dev),
            refl_offset=torch.empty(self.n_crystals + 1, dtype=torch.int64, device=dev))

    def new_peaks(self) -> Peaks:
        n = max(self.refl_capacity, 1)
        dev = self.device
        return Peaks(
            two_theta=torch.empty(n, dtype=torch.float64, device=dev),
            intensity=torch.empty(n, dtype=torch.float64, device=dev),
            scaled=torch.empty(n, dtype=torch.float64, device=dev),
            mult=torch.empty(n, dtype=torch.int32, device=dev), first=torch.empty(n, dtype=torch.int64, device=dev),
            perm=torch.empty(n, dtype=torch.int64, device=dev),
            peak_offset=torch.empty(self.n_crystals + 1, dtype=torch.int64, device=dev))

    def new_sf(self):
        n = max(self.refl_capacity, 1)
        dt = torch.float32 if self.precision == "mixed" else torch.float64
        return (torch.empty(n, dtype=dt, device=self.device), torch.empty(n, dtype=dt, device=self.device),
                torch.empty(n, dtype=torch.float64, device=self.device))

    # ---- the C calls --------------------------------------------------------

    def enumerate(self, refl: Optional[Reflections] = None) -> Reflections:
        refl = refl or self.new_reflections()
        capi.xrd_enumerate_hkl(self.handle, self.ws, refl.c())
        return refl

    def structure_factors(self, refl: Reflections, out=None):
        A, B, I = out or self.new_sf()
        capi.xrd_structure_factors(self.handle, self.ws, refl.c(), A.data_ptr(), B.data_ptr(), I.data_ptr())
        return A, B, I

    def autotune(self, refl: Reflections):
        """Time the structure-factor split candidates on ``refl`` (enumerated on
        this batch), at each tile shape unless the batch fixed one, and keep the
        fastest; returns (forward, adjoint) thresholds and, for sf_method
        "auto", the atom threshold of the recurrence (else -1).  The chosen
        shape is ``sf_rpt``."""
        return capi.xrd_autotune(self.handle, self.ws, refl.c())

    @property
    def sf_rpt(self) -> int:
        """Current tile shape of the direct structure-factor sums (reflections per lane)."""
        return capi.xrd_batch_get_sf_rpt(self.handle)

    def preferred_orientation(self, refl: Reflections, I: torch.Tensor, hp, march_r) -> torch.Tensor:
        """March-Dollase texture applied to I in place; hp [n_crystals, 3]
        (hkl components) and march_r [n_crystals], arrays or tensors."""
        f64 = dict(dtype=torch.float64, device=self.device)
        self._hp = torch.as_tensor(np.asarray(hp, dtype=np.float64).reshape(self.n_crystals, 3), **f64).contiguous()
        self._mr = torch.as_tensor(np.asarray(march_r, dtype=np.float64).reshape(self.n_crystals), **f64).contiguous()
        capi.xrd_preferred_orientation(self.handle, self.ws, refl.c(), self._hp.data_ptr(), self._mr.data_ptr(),
                                       I.data_ptr())
        return I

    def pattern_caglioti(self, refl: Reflections, I: torch.Tensor, grid: Grid, U: float, V: float, W: float,
                         y=None, eta: float = 0.0) -> torch.Tensor:
        """Broadened pattern with widths FWHM^2 = U tan^2 + V tan + W (grid.sigma
        unused) and pseudo-Voigt profiles of Lorentzian share eta (0: Gaussian)."""
        if y is None:
            y = torch.empty(self.n_crystals, grid.n_points, dtype=torch.float64, device=self.device)
        capi.xrd_pattern_caglioti(self.handle, self.ws, refl.c(), I.data_ptr(), grid.c(), U, V, W, y.data_ptr(), eta)
        return y

    def noise(self, y: torch.Tensor, seed: int, rel: float, abs_: float) -> torch.Tensor:
        """Seeded noise added to the broadened patterns y in place."""
        if y.dtype != torch.float64 or not y.is_contiguous() or y.shape[0] != self.n_crystals:
            raise ValueError("y must be a contiguous float64 [n_crystals, n_points] tensor")
        capi.xrd_pattern_noise(self.handle, y.shape[1], seed, rel, abs_, y.data_ptr())
        return y

    def families(self, refl: Reflections, peaks: Peaks, rule: int = 0):
        """Families of equivalent reflections per peak (rule 0: indices, 1: lattice).
        Returns (n_families [peak_cap] int32, family_of [refl_cap] int32,
        family_label [refl_cap] int64, family_mult [refl_cap] int32)."""
        dev, pc, rc = self.device, max(self.sizes.peak_capacity, 1), max(self.sizes.refl_capacity, 1)
        out = (torch.zeros(pc, dtype=torch.int32, device=dev), torch.full((rc,), -1, dtype=torch.int32, device=dev),
               torch.full((rc,), -1, dtype=torch.int64, device=dev), torch.zeros(rc, dtype=torch.int32, device=dev))
        capi.xrd_peak_families(self.handle, self.ws, refl.c(), peaks.c(), rule, *(t.data_ptr() for t in out))
        return out

    def merge(self, refl: Reflections, I: torch.Tensor, peaks: Optional[Peaks] = None) -> Peaks:
        peaks = peaks or self.new_peaks()
        capi.xrd_merge_peaks(self.handle, self.ws, refl.c(), I.data_ptr(), peaks.c())
        return peaks

    def pattern_forward(self, refl: Reflections, I: torch.Tensor, grid: Grid, y=None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.n_crystals, grid.n_points, dtype=torch.float64, device=self.device)
        capi.xrd_pattern_forward(self.handle, self.ws, refl.c(), I.data_ptr(), grid.c(), y.data_ptr())
        return y

    def new_grads(self):
        n = max(self.batch.n_atoms, 1)
        return (torch.empty(n, 3, dtype=torch.float64, device=self.device),
                torch.empty(n, dtype=torch.float64, device=self.device),
                torch.empty(max(self.n_crystals, 1), 6, dtype=torch.float64, device=self.device))

    def pattern_backward(self, refl: Reflections, grid: Grid, dy: torch.Tensor, out=None):
        if dy.dtype != torch.float64 or not dy.is_contiguous():
            dy = dy.to(torch.float64).contiguous()
        dfrac, dbfac, dlat = out or self.new_grads()
        capi.xrd_pattern_backward(self.handle, self.ws, refl.c(), grid.c(), dy.data_ptr(), dfrac.data_ptr(),
                                  dbfac.data_ptr(), dlat.data_ptr())
        return dfrac[: self.batch.n_atoms], dbfac[: self.batch.n_atoms], dlat[: self.n_crystals]

    def read_counts(self, refl: Optional[Reflections] = None, peaks: Optional[Peaks] = None):
        ro = np.zeros(self.n_crystals + 1, np.int64) if refl is not None else None
        po = np.zeros(self.n_crystals + 1, np.int64) if peaks is not None else None
        capi.xrd_read_counts(self.handle, refl.c() if refl is not None else None,
                             peaks.c() if peaks is not None else None,
                             ro.ctypes.data if ro is not None else None, po.ctypes.data if po is not None else None)
        return ro, po


@dataclasses.dataclass
class PatternResult:
    """Host copy of a batch's forward pipeline (CSR over crystals)."""

    refl_offset: np.ndarray
    hkl: np.ndarray
    q: np.ndarray
    two_theta: np.ndarray
    lp: np.ndarray
    A: np.ndarray
    B: np.ndarray
    I: np.ndarray
    peak_offset: np.ndarray
    pk_two_theta: np.ndarray
    pk_intensity: np.ndarray
    pk_scaled: np.ndarray
    pk_mult: np.ndarray
    pk_first: np.ndarray
    perm: np.ndarray
    # families of equivalent reflections (only with a family rule): per peak
    # their number; at position first + f, family f's label (reflection
    # index) and multiplicity
    fam_n: Optional[np.ndarray] = None
    fam_label: Optional[np.ndarray] = None
    fam_mult: Optional[np.ndarray] = None

    def crystal(self, c):
        r0, r1 = int(self.refl_offset[c]), int(self.refl_offset[c + 1])
        p0, p1 = int(self.peak_offset[c]), int(self.peak_offset[c + 1])
        return slice(r0, r1), slice(p0, p1)


def simulate(batch: CrystalBatch, precision: str = "mixed", friedel: Optional[bool] = None,
             rel_threshold: float = 0.0, device="cuda", autotune: bool = False,
             family_rule: Optional[int] = None, sf_method: str = "direct", sf_rpt: int = 0) -> PatternResult:
    """Enumerate, structure factors, merge for every crystal; host arrays back.
    With ``autotune`` the structure-factor tile shape and split are tuned on
    the enumerated reflections first; with a ``family_rule`` (0: indices, 1:
    lattice) the peaks' families of equivalent reflections come back too."""
    xb = XrdBatch(batch, precision=precision, friedel=friedel, rel_threshold=rel_threshold, device=device,
                  sf_method=sf_method, sf_rpt=sf_rpt)
    refl = xb.enumerate()
    if autotune:
        xb.autotune(refl)
    A, B, I = xb.structure_factors(refl)
    pk = xb.merge(refl, I)
    fam = xb.families(refl, pk, family_rule) if family_rule is not None else None
    ro, po = xb.read_counts(refl, pk)
    n, m = int(ro[-1]), int(po[-1])
    cpu = lambda t, k: t[:k].cpu().numpy()
    extra = {} if fam is None else dict(fam_n=cpu(fam[0], m), fam_label=cpu(fam[2], n), fam_mult=cpu(fam[3], n))
    hkl = np.stack([cpu(refl.h, n), cpu(refl.k, n), cpu(refl.l, n)], axis=1).astype(np.int32)
    return PatternResult(refl_offset=ro, hkl=hkl, q=cpu(refl.q, n), two_theta=cpu(refl.two_theta, n),
                         lp=cpu(refl.lp, n), A=cpu(A, n).astype(np.float64), B=cpu(B, n).astype(np.float64),
                         I=cpu(I, n), peak_offset=po, pk_two_theta=cpu(pk.two_theta, m),
                         pk_intensity=cpu(pk.intensity, m), pk_scaled=cpu(pk.scaled, m), pk_mult=cpu(pk.mult, m),
                         pk_first=cpu(pk.first, m), perm=cpu(pk.perm, n), **extra)


class _Slot:
    """A planned batch with its reflection and structure-factor buffers, kept
    between calls of the differentiable pattern on the same inputs."""

    def __init__(self, xb, lattice):
        self.xb = xb
        self.refl = xb.new_reflections()
        self.sf = xb.new_sf()
        self.lattice = lattice.copy()
        self.busy = False  # a forward's state awaits its backward
        self.gen = 0       # forward calls served


# batches of the differentiable pattern, reused across calls: per (batch
# object, precision, friedel, grid size, device) a few slots
_POOL = {}
_POOL_SLOTS = 2


def _slot_for(spec, frac, bfac, lat, needs_grad):
    """A planned batch for this call: a free pooled one (its frac and B
    refreshed in place, its cells changed in place when the search boxes
    allow), or a new one."""
    batch, grid = spec["batch"], spec["grid"]
    key = (id(batch), spec["precision"], spec["friedel"], int(grid.n_points), str(frac.device))
    slots = [s for s in _POOL.get(key, []) if s.xb.batch is batch]
    _POOL[key] = slots
    for slot in slots:
        if slot.busy:
            continue
        xb = slot.xb
        if not np.array_equal(slot.lattice, lat):
            lat_c = np.ascontiguousarray(lat, dtype=np.float64)
            if capi.xrd_batch_set_lattice(xb.handle, lat_c.ctypes.data, xb.ws) != capi.XRD_OK:
                continue  # a cell outgrew its search box: plan anew below
            slot.lattice = lat_c.copy()
        xb.frac.copy_(frac.detach().to(torch.float64))
        xb.bfac.copy_(bfac.detach().to(torch.float64))
        break
    else:
        xb = XrdBatch(batch, precision=spec["precision"], friedel=spec["friedel"], device=frac.device,
                      frac=frac.detach().to(torch.float64).clone().contiguous(),
                      bfac=bfac.detach().to(torch.float64).clone().contiguous(), lattice=lat,
                      grid_capacity=grid.n_points, keep_sf_derivs=True)
        slot = _Slot(xb, lat)
        if len(slots) < _POOL_SLOTS:
            slots.append(slot)
    slot.gen += 1
    slot.busy = needs_grad
    return slot


class _PatternFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frac, lattice, bfac, spec):
        lat = lattice.detach().to("cpu", torch.float64).numpy()
        slot = _slot_for(spec, frac, bfac, lat, any(ctx.needs_input_grad[:3]))
        xb = slot.xb
        xb.enumerate(slot.refl)
        _, _, I = xb.structure_factors(slot.refl, slot.sf)
        y = xb.pattern_forward(slot.refl, I, spec["grid"])
        ctx.slot, ctx.gen, ctx.grid = slot, slot.gen, spec["grid"]
        ctx.lat_device, ctx.lat_dtype = lattice.device, lattice.dtype
        return y

    @staticmethod
    def backward(ctx, dy):
        slot = ctx.slot
        if slot.gen != ctx.gen:
            raise RuntimeError("the pattern's forward state was reused by a later call; call backward before "
                               "evaluating the pattern again")
        dfrac, dbfac, dlat = slot.xb.pattern_backward(slot.refl, ctx.grid, dy)
        dfrac, dbfac, dlat = dfrac.clone(), dbfac.clone(), dlat.clone()
        slot.busy = False
        return dfrac, dlat.to(ctx.lat_device, ctx.lat_dtype), dbfac, None


def xrd_pattern(frac: torch.Tensor, lattice: torch.Tensor, bfac: torch.Tensor, batch: CrystalBatch, grid: Grid,
                precision: str = "mixed", friedel: Optional[bool] = None) -> torch.Tensor:
    """Differentiable Gaussian-broadened pattern [n_crystals, n_points].

    ``frac`` [N, 3] and ``bfac`` [N] are device tensors, ``lattice``
    [n_crystals, 6] any tensor (read on the host to plan the batch); species,
    occupancies, scattering factors, wavelength and the enumeration range come
    from ``batch`` (whose 2theta range should cover the grid widened by the
    window).  Gradients flow to frac, lattice (per degree for angles) and bfac
    through the library's adjoint; the reflection set is held fixed.  The
    planned batch and its device buffers are kept between calls on the same
    ``batch`` (a new cell takes the old plan when its search box allows), so
    a refinement loop does not plan and allocate on every step; call
    backward before the pattern of the same inputs is evaluated again."""
    spec = {"batch": batch, "grid": grid, "precision": precision,
            "friedel": (precision == "mixed") if friedel is None else friedel}
    return _PatternFn.apply(frac, lattice, bfac, spec)
