"""Calculator front-end over plain arrays, with X-ray tube doublets.

The paper's calculator (Section 2, Fig. 1) takes a structure (lattice,
fractional coordinates, species, occupancies, thermal factors), a wavelength,
a 2theta range and a ``scaled`` flag, and returns the peaks with their 2theta,
intensity, hkl lists and multiplicities.  ``get_pattern`` offers that call
for one structure given as arrays, ``get_patterns`` for a whole
``CrystalBatch``; both run on the GPU library (enumeration, structure
factors, sort and merge, and the combination of the lines' peaks).  A
wavelength is a number in Angstrom or the name of an emission line; a doublet name ("CuKa12", "MoKa12") computes the K-alpha1
and K-alpha2 lines separately, weights K-alpha2 by ``KA2_RATIO`` and lists the
peaks of both lines in one 2theta-ordered pattern, scaled together.
``broadened_pattern`` does the same on a grid (the sum of the two lines'
broadened patterns).

A peak's ``hkls`` lists its families of symmetry-equivalent reflections
(paper, Section 2: grouping of equivalent reflections; Section 3: each entry
an hkl with a multiplicity), each as {"hkl": label, "multiplicity": m}, the
label being the family's lexicographically largest member; ``family_rule``
"indices" groups equal multisets of absolute indices (4-index form on
hexagonal lattices), "lattice" groups reflections related by a point
operation of the lattice.  On a hexagonal lattice (a = b, alpha = beta =
90, gamma = 120 degrees) family labels are written as Miller-Bravais
4-tuples (h, k, -(h + k), l), as the Python calculator the paper targets
writes them.  ``members`` lists every member reflection (Friedel mates
included) in (2theta, h, k, l) order.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Union

import numpy as np

from .synth import CrystalBatch

# K-alpha1 and K-alpha2 emission lines (Angstrom; Deslattes et al., Rev. Mod.
# Phys. 75, 35 (2003)), K-alpha2 weighted by KA2_RATIO.  The single-line
# names "CuKa" and "MoKa" are the conventional single K-alpha wavelengths
# 1.54184 and 0.71073 Angstrom (the values the synthetic workloads use), not
# computed from the doublet.
KA2_RATIO = 0.5
_LINES = {"Cu": (1.5405929, 1.5444274), "Mo": (0.7093171, 0.7135900)}
_SINGLE = {"Cu": 1.54184, "Mo": 0.71073}
WAVELENGTHS = {}
for _el, (_a1, _a2) in _LINES.items():
    WAVELENGTHS[_el + "Ka1"] = _a1
    WAVELENGTHS[_el + "Ka2"] = _a2
    WAVELENGTHS[_el + "Ka"] = _SINGLE[_el]


def lines_of(wavelength: Union[float, str]):
    """[(wavelength in Angstrom, intensity weight, line label)] of a wavelength spec."""
    if isinstance(wavelength, str):
        if wavelength.endswith("Ka12") and wavelength[:-4] in _LINES:
            a1, a2 = _LINES[wavelength[:-4]]
            return [(a1, 1.0, "a1"), (a2, KA2_RATIO, "a2")]
        if wavelength in WAVELENGTHS:
            return [(WAVELENGTHS[wavelength], 1.0, "")]
        raise ValueError(f"unknown wavelength {wavelength!r}; known: {sorted(WAVELENGTHS)} and "
                         f"{[e + 'Ka12' for e in _LINES]}")
    lam = float(wavelength)
    if not lam > 0.0:
        raise ValueError("wavelength must be > 0")
    return [(lam, 1.0, "")]


@dataclasses.dataclass
class DiffractionPattern:
    """Peaks of one structure in ascending 2theta."""

    x: np.ndarray        # 2theta (degrees)
    y: np.ndarray        # intensity (0-100 when scaled)
    mult: np.ndarray     # member reflections per peak (the sum of its family multiplicities)
    d_hkls: np.ndarray   # interplanar spacing (Angstrom)
    hkls: list           # per peak: its families, [{"hkl": (h, k, l) or (h, k, i, l), "multiplicity": m}, ...]
    line: np.ndarray     # per peak: emission line label ("" for a single line)
    members: list        # per peak: (h, k, l) of its members, in (2theta, h, k, l) order


def structure_batch(lattice: Sequence[float], frac, species, sf_coeff, occ=None, bfac=None,
                    two_theta_range=(0.0, 90.0), merge_tol: float = 1e-5) -> CrystalBatch:
    """A one-crystal CrystalBatch from plain arrays (validated here)."""
    lat = np.asarray(lattice, dtype=np.float64).reshape(6)
    frac = np.asarray(frac, dtype=np.float64).reshape(-1, 3)
    n = frac.shape[0]
    species = np.asarray(species, dtype=np.int32).reshape(n)
    coeff = np.asarray(sf_coeff, dtype=np.float64).reshape(-1, 9)
    occ = np.ones(n) if occ is None else np.asarray(occ, dtype=np.float64).reshape(n)
    bfac = np.zeros(n) if bfac is None else np.asarray(bfac, dtype=np.float64).reshape(n)
    if n and (species.min() < 0 or species.max() >= coeff.shape[0]):
        raise ValueError("species index outside the coefficient table")
    t0, t1 = (float(two_theta_range[0]), float(two_theta_range[1]))
    if not (0.0 <= t0 < t1 < 180.0):
        raise ValueError("two_theta_range must satisfy 0 <= min < max < 180")
    return CrystalBatch("structure", lat[None, :].copy(), np.array([0, n], np.int64), frac, species, occ, bfac,
                        coeff, 1.0, np.array([t0]), np.array([t1]), merge_tol)


FAMILY_RULES = {"indices": 0, "lattice": 1}


def is_hexagonal(lattice, tol: float = 1e-6) -> bool:
    """a = b, alpha = beta = 90, gamma = 120 degrees (relative / absolute tolerance)."""
    a, b, _, al, be, ga = (float(v) for v in np.asarray(lattice, dtype=np.float64).reshape(6))
    return abs(a - b) <= tol * max(a, b) and abs(al - 90.0) <= 1e3 * tol and abs(be - 90.0) <= 1e3 * tol \
        and abs(ga - 120.0) <= 1e3 * tol


def _label(hkl, hexagonal: bool):
    h, k, l = (int(v) for v in hkl)
    return (h, k, -(h + k), l) if hexagonal else (h, k, l)


def _line_peaks(batch: CrystalBatch, lam: float, precision: str, device, rule: int):
    """One emission line on the GPU: enumeration, structure factors, merge and
    families; the batch, its reflections, peaks and families (device)."""
    from .api import XrdBatch
    xb = XrdBatch(dataclasses.replace(batch, wavelength=lam), precision=precision, device=device,
                  forward_only=True)
    refl = xb.enumerate()
    _, _, I = xb.structure_factors(refl)
    pk = xb.merge(refl, I)
    fam = xb.families(refl, pk, rule)
    return xb, refl, pk, fam


def get_patterns(batch: CrystalBatch, wavelength: Union[float, str] = "CuKa", scaled: bool = True,
                 precision: str = "mixed", device="cuda", family_rule: str = "indices") -> list:
    """Peaks of every crystal of ``batch`` (its own wavelength is replaced by
    ``wavelength``), one DiffractionPattern per crystal.  The lines' peaks are
    combined on the GPU (xrd_combine_lines: weights, joint 0-100 scale,
    interplanar spacings); the host only gathers each peak's hkl lists."""
    import ctypes
    import torch
    from . import capi
    if family_rule not in FAMILY_RULES:
        raise ValueError(f"family_rule must be one of {sorted(FAMILY_RULES)}")
    lines = lines_of(wavelength)
    runs = [_line_peaks(batch, lam, precision, device, FAMILY_RULES[family_rule]) for lam, _, _ in lines]
    n_c = batch.n_crystals
    dev = runs[0][0].device
    cap = max(sum(xb.refl_capacity for xb, _, _, _ in runs), 1)
    e = lambda dt: torch.empty(cap, dtype=dt, device=dev)
    out_t = dict(two_theta=e(torch.float64), intensity=e(torch.float64), scaled=e(torch.float64),
                 mult=e(torch.int32), d=e(torch.float64), line=e(torch.int32), source=e(torch.int64),
                 peak_offset=torch.empty(n_c + 1, dtype=torch.int64, device=dev))
    out = capi.xrd_line_peaks(*(out_t[k].data_ptr() for k in ("two_theta", "intensity", "scaled", "mult", "d",
                                                               "line", "source", "peak_offset")))
    pks = [pk.c() for _, _, pk, _ in runs]  # kept alive across the call
    ln = [capi.xrd_line(ctypes.pointer(pc), refl.q.data_ptr(), float(w))
          for pc, (_, refl, _, _), (_, w, _) in zip(pks, runs, lines)]
    stream = runs[0][0].stream
    for xb, _, _, _ in runs[1:]:
        stream.wait_stream(xb.stream)
    with torch.cuda.stream(stream):
        capi.xrd_combine_lines(n_c, ln[0], ln[1] if len(ln) > 1 else None, out, stream.cuda_stream)
    torch.cuda.synchronize(dev)
    po = out_t["peak_offset"].cpu().numpy()
    m = int(po[-1])
    host = {k: out_t[k][:m].cpu().numpy() for k in ("two_theta", "intensity", "scaled", "mult", "d", "line",
                                                    "source")}
    # per line, what the hkl lists need: members (perm), indices and families
    per_line = []
    for xb, refl, pk, fam in runs:
        ro, lpo = xb.read_counts(refl, pk)
        n, mp = int(ro[-1]), int(lpo[-1])
        cpu = lambda t, k: t[:k].cpu().numpy()
        hkl = np.stack([cpu(refl.h, n), cpu(refl.k, n), cpu(refl.l, n)], axis=1).astype(np.int32)
        per_line.append(dict(hkl=hkl, perm=cpu(pk.perm, n), first=cpu(pk.first, mp), mult=cpu(pk.mult, mp),
                             fam_n=cpu(fam[0], mp), fam_label=cpu(fam[2], n), fam_mult=cpu(fam[3], n)))
    labels = np.array([label for _, _, label in lines])
    y_all = host["scaled"] if scaled else host["intensity"]
    # each combined peak's members and families, gathered per line with array
    # operations and turned into Python objects in bulk
    hexa = np.array([is_hexagonal(batch.lattice[c]) for c in range(n_c)], dtype=bool)
    peak_crystal = np.repeat(np.arange(n_c), np.diff(po))
    members_of = [None] * m
    families_of = [None] * m

    def runs_of(start, count):
        # start[p] + 0 .. count[p] - 1 for every p, concatenated
        total = int(count.sum())
        base = np.repeat(start - (np.cumsum(count) - count), count)
        return base + np.arange(total, dtype=np.int64)

    for li, L in enumerate(per_line):
        sel = np.nonzero(host["line"] == li)[0]
        if len(sel) == 0:
            continue
        src = host["source"][sel]
        f = L["first"][src].astype(np.int64)
        mlt = L["mult"][src].astype(np.int64)
        rows = list(map(tuple, L["hkl"][L["perm"][runs_of(f, mlt)]].tolist()))
        offs = np.concatenate([[0], np.cumsum(mlt)]).tolist()
        nf = L["fam_n"][src].astype(np.int64)
        fpos = runs_of(f, nf)
        fh = L["hkl"][L["fam_label"][fpos]].astype(np.int64)
        hx = np.repeat(hexa[peak_crystal[sel]], nf)
        fm_mult = L["fam_mult"][fpos].tolist()
        fl = [_label(r, x) for r, x in zip(fh.tolist(), hx.tolist())]
        foffs = np.concatenate([[0], np.cumsum(nf)]).tolist()
        for j, p in enumerate(sel.tolist()):
            members_of[p] = rows[offs[j]:offs[j + 1]]
            families_of[p] = [{"hkl": fl[q], "multiplicity": int(fm_mult[q])} for q in range(foffs[j], foffs[j + 1])]
    result = []
    for c in range(n_c):
        p0, p1 = int(po[c]), int(po[c + 1])
        result.append(DiffractionPattern(x=host["two_theta"][p0:p1].copy(), y=y_all[p0:p1].copy(),
                                         mult=host["mult"][p0:p1].copy(), d_hkls=host["d"][p0:p1].copy(),
                                         hkls=families_of[p0:p1], line=labels[host["line"][p0:p1]],
                                         members=members_of[p0:p1]))
    return result


def get_pattern(lattice, frac, species, sf_coeff, occ=None, bfac=None, wavelength: Union[float, str] = "CuKa",
                scaled: bool = True, two_theta_range=(0.0, 90.0), merge_tol: float = 1e-5,
                precision: str = "mixed", device="cuda", family_rule: str = "indices") -> DiffractionPattern:
    """Peaks of one structure given as arrays: lattice (a, b, c, alpha, beta,
    gamma), fractional coordinates [N, 3], species rows of ``sf_coeff``
    ([S, 9]: a1..a4, b1..b4, c), occupancies and B factors (default 1 and 0)."""
    b = structure_batch(lattice, frac, species, sf_coeff, occ, bfac, two_theta_range, merge_tol)
    return get_patterns(b, wavelength, scaled, precision, device, family_rule)[0]


def broadened_pattern(batch: CrystalBatch, grid, wavelength: Union[float, str] = "CuKa",
                      precision: str = "mixed", device="cuda", widths: Optional[Sequence[float]] = None,
                      eta: float = 0.0):
    """[n_crystals, n_points] broadened pattern of ``batch`` on ``grid``
    (api.Grid): the weighted sum over the wavelength's emission lines.  With
    ``widths`` = (U, V, W) each line has the angle-dependent FWHM^2 = U tan^2
    + V tan + W (Caglioti) and a pseudo-Voigt profile of Lorentzian share
    ``eta``, instead of the grid's one Gaussian width."""
    if widths is None and eta != 0.0:
        raise ValueError("eta needs widths (U, V, W)")
    import torch
    from .api import XrdBatch
    y = None
    for lam, weight, _ in lines_of(wavelength):
        xb = XrdBatch(dataclasses.replace(batch, wavelength=lam), precision=precision, device=device,
                      grid_capacity=grid.n_points)
        refl = xb.enumerate()
        _, _, I = xb.structure_factors(refl)
        if widths is None:
            part = xb.pattern_forward(refl, I, grid)
        else:
            U, V, W = (float(v) for v in widths)
            part = xb.pattern_caglioti(refl, I, grid, U, V, W, eta=eta)
        y = weight * part if y is None else y + weight * part
    torch.cuda.synchronize()
    return y
