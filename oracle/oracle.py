"""ctypes front end of the FP64 oracle (test infrastructure only).

Each function wraps one routine of ``xrd_oracle.c``; ``pattern`` and
``pattern_batch`` return the whole pipeline (enumerate, structure factors,
Lorentz-polarisation, intensity, sort, merge, scaling) of one crystal or of a
batch; ``broadened`` and ``loss`` give the Gaussian-broadened pattern and the
mean-squared-error loss whose gradients the library's adjoint must match.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xrd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

__all__ = [
    "build", "cell", "q_of", "two_theta", "lp", "lp_many", "fsc", "enumerate_hkl",
    "structure_factors", "sort_order", "merge", "broaden", "OracleCrystal",
    "pattern", "pattern_batch", "broadened", "loss", "march_dollase", "splitmix64", "gauss", "noise",
    "broaden_caglioti", "FAM_INDICES", "FAM_LATTICE", "is_hexagonal", "lattice_ops", "peak_families",
]

FAM_INDICES = 0
FAM_LATTICE = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (double precision, FMA contraction off)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class _Crystal(C.Structure):
    _fields_ = [
        ("n_refl", C.c_long), ("n_peaks", C.c_long), ("amb_bound", C.c_long), ("amb_gap", C.c_long),
        ("hkl", C.POINTER(C.c_int)),
        ("q", C.POINTER(C.c_double)), ("tt", C.POINTER(C.c_double)), ("lp", C.POINTER(C.c_double)),
        ("fr", C.POINTER(C.c_double)), ("fi", C.POINTER(C.c_double)), ("absw", C.POINTER(C.c_double)),
        ("inten", C.POINTER(C.c_double)),
        ("perm", C.POINTER(C.c_long)),
        ("pk_tt", C.POINTER(C.c_double)), ("pk_i", C.POINTER(C.c_double)), ("pk_y", C.POINTER(C.c_double)),
        ("pk_mult", C.POINTER(C.c_int)),
        ("pk_first", C.POINTER(C.c_long)),
        ("status", C.c_int),
    ]


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.orc_cell.argtypes = [_dp, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_cell.restype = C.c_int
        lib.orc_q.argtypes = [_dp, C.c_int, C.c_int, C.c_int]
        lib.orc_q.restype = C.c_double
        lib.orc_two_theta.argtypes = [C.c_double, C.c_double]
        lib.orc_two_theta.restype = C.c_double
        lib.orc_lp.argtypes = [C.c_double]
        lib.orc_lp.restype = C.c_double
        lib.orc_lp_many.argtypes = [C.c_long, _dp, _dp]
        lib.orc_lp_many.restype = None
        lib.orc_fsc.argtypes = [_dp, C.c_double]
        lib.orc_fsc.restype = C.c_double
        lib.orc_enumerate.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_long,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_long)]
        lib.orc_enumerate.restype = C.c_long
        lib.orc_structure_factors.argtypes = [C.c_long, _ip, _dp, C.c_long, _dp, _ip, _dp, _dp, _dp,
                                              _dp, _dp, _dp]
        lib.orc_structure_factors.restype = None
        lib.orc_sort.argtypes = [C.c_long, _dp, _ip, _lp]
        lib.orc_sort.restype = None
        lib.orc_merge.argtypes = [C.c_long, _dp, _dp, C.c_double, _dp, _dp, _ip, _lp,
                                  C.POINTER(C.c_long)]
        lib.orc_merge.restype = C.c_long
        lib.orc_broaden.argtypes = [C.c_long, _dp, _dp, C.c_double, C.c_double, C.c_long,
                                    C.c_double, C.c_double, _dp]
        lib.orc_broaden.restype = None
        lib.orc_pattern.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_long, _dp, _ip, _dp, _dp, _dp, C.POINTER(_Crystal)]
        lib.orc_pattern.restype = None
        lib.orc_pattern_batch.argtypes = [C.c_long, _dp, _lp, _dp, _ip, _dp, _dp, _dp, C.c_double,
                                          _dp, _dp, C.c_double, C.c_double, C.c_int,
                                          C.POINTER(_Crystal)]
        lib.orc_pattern_batch.restype = None
        lib.orc_free_crystal.argtypes = [C.POINTER(_Crystal)]
        lib.orc_free_crystal.restype = None
        lib.orc_march_dollase.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, C.c_double]
        lib.orc_march_dollase.restype = C.c_double
        lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        lib.orc_splitmix64.restype = C.c_uint64
        lib.orc_gauss.argtypes = [C.c_uint64, C.c_uint64]
        lib.orc_gauss.restype = C.c_double
        lib.orc_noise.argtypes = [C.c_long, C.c_long, C.c_uint64, C.c_double, C.c_double, _dp]
        lib.orc_noise.restype = None
        lib.orc_broaden_caglioti.argtypes = [C.c_long, _dp, _dp, C.c_double, C.c_double, C.c_long, C.c_double,
                                             C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        lib.orc_broaden_caglioti.restype = None
        lib.orc_is_hexagonal.argtypes = [_dp]
        lib.orc_is_hexagonal.restype = C.c_int
        lib.orc_lattice_ops.argtypes = [_dp, C.c_long, _ip]
        lib.orc_lattice_ops.restype = C.c_long
        lib.orc_peak_families.argtypes = [_dp, C.c_int, C.c_long, _lp, _lp, _ip, _lp, _lp, _ip, _lp]
        lib.orc_peak_families.restype = C.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---- primitives ----------------------------------------------------------

def cell(lattice):
    """(G, G*, volume) of a cell as 6-vectors [11, 22, 33, 12, 13, 23], or None if invalid."""
    g = np.zeros(6)
    gs = np.zeros(6)
    vol = C.c_double()
    st = _get().orc_cell(_f64(lattice), g.ctypes.data, gs.ctypes.data, C.addressof(vol))
    return None if st else (g, gs, vol.value)


def q_of(gs, h, k, l):
    return _get().orc_q(_f64(gs), int(h), int(k), int(l))


def two_theta(q, wavelength):
    return _get().orc_two_theta(float(q), float(wavelength))


def lp(two_theta_deg):
    return _get().orc_lp(float(two_theta_deg))


def lp_many(two_theta_deg):
    """lp of every angle of an array."""
    tt = _f64(two_theta_deg).reshape(-1)
    out = np.zeros(max(len(tt), 1))
    _get().orc_lp_many(len(tt), tt if len(tt) else np.zeros(1), out)
    return out[:len(tt)]


def fsc(coeff, s2):
    return _get().orc_fsc(_f64(coeff), float(s2))


def enumerate_hkl(lattice, wavelength, tmin, tmax):
    """(hkl int32 [R, 3], q [R], 2theta [R], ambiguous-bound count), lexicographic order."""
    lib = _get()
    lat = _f64(lattice)
    n = lib.orc_enumerate(lat, wavelength, tmin, tmax, 0, None, None, None, None)
    if n < 0:
        raise ValueError("invalid cell or 2theta range")
    hkl = np.zeros((max(n, 1), 3), np.int32)
    q = np.zeros(max(n, 1))
    tt = np.zeros(max(n, 1))
    amb = C.c_long()
    lib.orc_enumerate(lat, wavelength, tmin, tmax, n, hkl.ctypes.data, q.ctypes.data,
                      tt.ctypes.data, C.byref(amb))
    return hkl[:n], q[:n], tt[:n], amb.value


def structure_factors(hkl, q, frac, species, occ, bfac, coeff):
    """(Re F, Im F, sum |w|) for each listed reflection."""
    hkl = _i32(hkl).reshape(-1, 3)
    nr = hkl.shape[0]
    fr = np.zeros(max(nr, 1))
    fi = np.zeros(max(nr, 1))
    aw = np.zeros(max(nr, 1))
    frac = _f64(frac).reshape(-1, 3)
    _get().orc_structure_factors(nr, hkl if nr else np.zeros((1, 3), np.int32), _f64(q) if nr else np.zeros(1),
                                 frac.shape[0], frac if frac.size else np.zeros((1, 3)),
                                 _i32(species) if len(species) else np.zeros(1, np.int32),
                                 _f64(occ) if len(occ) else np.zeros(1),
                                 _f64(bfac) if len(bfac) else np.zeros(1), _f64(coeff), fr, fi, aw)
    return fr[:nr], fi[:nr], aw[:nr]


def sort_order(tt, hkl):
    tt = _f64(tt)
    perm = np.zeros(max(len(tt), 1), np.int64)
    _get().orc_sort(len(tt), tt if len(tt) else np.zeros(1), _i32(hkl).reshape(-1, 3) if len(tt)
                    else np.zeros((1, 3), np.int32), perm)
    return perm[:len(tt)]


def merge(tt_sorted, i_sorted, tol):
    """Anchor-rule merge: (peak 2theta, peak I, mult, first, ambiguous count)."""
    n = len(tt_sorted)
    m = max(n, 1)
    pt, pi, pm, pf = np.zeros(m), np.zeros(m), np.zeros(m, np.int32), np.zeros(m, np.int64)
    amb = C.c_long()
    ts = _f64(tt_sorted) if n else np.zeros(1)
    is_ = _f64(i_sorted) if n else np.zeros(1)
    np_ = _get().orc_merge(n, ts, is_, float(tol), pt, pi, pm, pf, C.byref(amb))
    return pt[:np_], pi[:np_], pm[:np_], pf[:np_], amb.value


def broaden(tt, inten, t0, dt, npts, sigma, window):
    y = np.zeros(npts)
    n = len(tt)
    _get().orc_broaden(n, _f64(tt) if n else np.zeros(1), _f64(inten) if n else np.zeros(1),
                       float(t0), float(dt), int(npts), float(sigma), float(window), y)
    return y


# ---- whole patterns --------------------------------------------------------

@dataclasses.dataclass
class OracleCrystal:
    hkl: np.ndarray      # [R, 3] int32, enumeration order
    q: np.ndarray
    tt: np.ndarray
    lp: np.ndarray
    fr: np.ndarray
    fi: np.ndarray
    absw: np.ndarray
    inten: np.ndarray
    perm: np.ndarray     # [R] sorted order
    pk_tt: np.ndarray
    pk_i: np.ndarray
    pk_y: np.ndarray
    pk_mult: np.ndarray
    pk_first: np.ndarray
    amb_bound: int
    amb_gap: int

    @property
    def n_refl(self):
        return len(self.tt)


def _take(c: _Crystal) -> OracleCrystal:
    if c.status != 0:
        raise ValueError(f"oracle rejected the crystal (status {c.status})")
    n, p = c.n_refl, c.n_peaks

    def arr(ptr, cnt, dt, shape=None):
        if cnt == 0:
            return np.zeros(shape if shape else (0,), dt)
        a = np.ctypeslib.as_array(ptr, shape=(cnt,)).astype(dt, copy=True)
        return a.reshape(shape) if shape else a

    return OracleCrystal(
        hkl=arr(c.hkl, 3 * n, np.int32, (n, 3)), q=arr(c.q, n, np.float64),
        tt=arr(c.tt, n, np.float64), lp=arr(c.lp, n, np.float64), fr=arr(c.fr, n, np.float64),
        fi=arr(c.fi, n, np.float64), absw=arr(c.absw, n, np.float64),
        inten=arr(c.inten, n, np.float64), perm=arr(c.perm, n, np.int64),
        pk_tt=arr(c.pk_tt, p, np.float64), pk_i=arr(c.pk_i, p, np.float64),
        pk_y=arr(c.pk_y, p, np.float64), pk_mult=arr(c.pk_mult, p, np.int32),
        pk_first=arr(c.pk_first, p, np.int64), amb_bound=c.amb_bound, amb_gap=c.amb_gap)


def pattern(batch, c: int, threshold: float = 0.0) -> OracleCrystal:
    """Full pattern of crystal ``c`` of a synthetic batch."""
    lib = _get()
    sl = batch.atoms_of(c)
    na = sl.stop - sl.start
    out = _Crystal()
    frac = _f64(batch.frac[sl]) if na else np.zeros((1, 3))
    lib.orc_pattern(_f64(batch.lattice[c]), batch.wavelength, float(batch.two_theta_min[c]),
                    float(batch.two_theta_max[c]), batch.merge_tol, float(threshold), na, frac,
                    _i32(batch.species[sl]) if na else np.zeros(1, np.int32),
                    _f64(batch.occ[sl]) if na else np.zeros(1),
                    _f64(batch.bfac[sl]) if na else np.zeros(1), _f64(batch.sf_coeff), C.byref(out))
    try:
        return _take(out)
    finally:
        lib.orc_free_crystal(C.byref(out))


def pattern_batch(batch, threads: int = 1, threshold: float = 0.0, keep: bool = True):
    """Patterns of every crystal of a batch on ``threads`` OpenMP threads.

    With keep=False the results are freed without conversion (timing use)."""
    lib = _get()
    nc = batch.n_crystals
    outs = (_Crystal * max(nc, 1))()
    na = batch.n_atoms
    lib.orc_pattern_batch(nc, _f64(batch.lattice), np.ascontiguousarray(batch.atom_offset, np.int64),
                          _f64(batch.frac) if na else np.zeros((1, 3)),
                          _i32(batch.species) if na else np.zeros(1, np.int32),
                          _f64(batch.occ) if na else np.zeros(1),
                          _f64(batch.bfac) if na else np.zeros(1), _f64(batch.sf_coeff),
                          batch.wavelength, _f64(batch.two_theta_min), _f64(batch.two_theta_max),
                          batch.merge_tol, float(threshold), int(threads), outs)
    res = []
    try:
        for c in range(nc):
            if keep:
                res.append(_take(outs[c]))
            elif outs[c].status != 0:
                raise ValueError(f"oracle rejected crystal {c}")
    finally:
        for c in range(nc):
            lib.orc_free_crystal(C.byref(outs[c]))
    return res


def broadened(batch, c: int, t0: float, dt: float, npts: int, sigma: float, window: float):
    """Gaussian-broadened pattern of crystal ``c``: every reflection in the
    crystal's enumeration range contributes, unmerged, with its own intensity."""
    hkl, q, tt, _ = enumerate_hkl(batch.lattice[c], batch.wavelength,
                                  float(batch.two_theta_min[c]), float(batch.two_theta_max[c]))
    sl = batch.atoms_of(c)
    fr, fi, _ = structure_factors(hkl, q, batch.frac[sl], batch.species[sl], batch.occ[sl],
                                  batch.bfac[sl], batch.sf_coeff)
    inten = (fr * fr + fi * fi) * lp_many(tt)
    return broaden(tt, inten, t0, dt, npts, sigma, window)


def loss(batch, targets, t0, dt, npts, sigma, window, crystals=None):
    """Mean over the listed crystals and grid points of (y - target)^2.

    ``targets`` is indexed by crystal; ``crystals`` defaults to all."""
    crystals = range(batch.n_crystals) if crystals is None else crystals
    tot, cnt = 0.0, 0
    for c in crystals:
        y = broadened(batch, c, t0, dt, npts, sigma, window)
        d = y - targets[c]
        tot += float(np.dot(d, d))
        cnt += npts
    return tot / cnt


# ---- augmentation of ML training patterns -----------------------------------

def march_dollase(gs, h, k, l, hp, r):
    """March-Dollase preferred-orientation factor of reflection (h, k, l)."""
    return _get().orc_march_dollase(_f64(gs), int(h), int(k), int(l), _f64(hp), float(r))


def splitmix64(seed, j):
    """Output j (>= 1) of SplitMix64 seeded with ``seed``."""
    return int(_get().orc_splitmix64(int(seed) & (2**64 - 1), int(j) & (2**64 - 1)))


def gauss(seed, n):
    """Standard normal variate n of stream ``seed``."""
    return _get().orc_gauss(int(seed) & (2**64 - 1), int(n))


def noise(y, seed, rel, abs_):
    """y [n_c, n_pts] with noise added (a new array)."""
    out = np.array(y, dtype=np.float64, order="C", copy=True)
    n_c, n_pts = out.shape
    _get().orc_noise(n_c, n_pts, int(seed) & (2**64 - 1), float(rel), float(abs_), out)
    return out


def broaden_caglioti(tt, inten, t0, dt, npts, U, V, W, window, eta=0.0):
    """Broadened pattern with Caglioti widths FWHM^2 = U tan^2 + V tan + W and
    pseudo-Voigt profiles of Lorentzian share eta (0: Gaussian)."""
    y = np.zeros(npts)
    n = len(tt)
    _get().orc_broaden_caglioti(n, _f64(tt) if n else np.zeros(1), _f64(inten) if n else np.zeros(1),
                                float(t0), float(dt), int(npts), float(U), float(V), float(W), float(eta),
                                float(window), y)
    return y


def is_hexagonal(lattice) -> bool:
    return bool(_get().orc_is_hexagonal(_f64(lattice)))


def lattice_ops(lattice):
    """Point operations of the lattice (integer matrices, entries in {-1, 0, 1})."""
    ops = np.zeros((48, 9), dtype=np.int32)
    n = _get().orc_lattice_ops(_f64(lattice), 48, ops)
    if n < 0:
        raise ValueError("invalid cell or more than 48 operations")
    return ops[:n].reshape(n, 3, 3).copy()


def peak_families(lattice, rule, first, mult, hkl):
    """Families of one crystal's peaks.  hkl [n, 3] in peak member order; peak p
    owns positions first[p] .. first[p] + mult[p] - 1.  Returns (fam [n],
    n_fam [n_peaks], label [n, 3], fam_mult [n]); family f of peak p sits at
    position first[p] + f of label and fam_mult."""
    first = np.ascontiguousarray(first, dtype=np.int64)
    mult = np.ascontiguousarray(mult, dtype=np.int64)
    hkl = np.ascontiguousarray(np.asarray(hkl).reshape(-1, 3), dtype=np.int32)
    n = max(len(hkl), 1)
    fam = np.full(n, -1, dtype=np.int64)
    n_fam = np.zeros(max(len(first), 1), dtype=np.int64)
    label = np.zeros((n, 3), dtype=np.int32)
    fam_mult = np.zeros(n, dtype=np.int64)
    rc = _get().orc_peak_families(_f64(lattice), int(rule), len(first), first if len(first) else np.zeros(1, np.int64),
                                  mult if len(mult) else np.zeros(1, np.int64), hkl if len(hkl) else np.zeros((1, 3), np.int32),
                                  fam, n_fam, label, fam_mult)
    if rc:
        raise ValueError("invalid cell or rule")
    m = len(hkl)
    return fam[:m], n_fam[:len(first)], label[:m], fam_mult[:m]
