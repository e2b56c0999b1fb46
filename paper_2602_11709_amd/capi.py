"""ctypes binding of libxrd.so: the C ABI of include/xrd.h, same names.

Argument marshalling only.  Every step of the pipeline runs in the library's
gfx950 kernels; importing this module fails loudly when the library has not
been built (``python -m paper_2602_11709_amd.build``).
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxrd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "xrd.h")

XRD_OK = 0
XRD_ERR_INVALID_ARG = -1
XRD_ERR_INVALID_CELL = -2
XRD_ERR_CAPACITY = -3
XRD_ERR_HIP = -4
XRD_ERR_UNSUPPORTED = -5
XRD_FP64 = 0
XRD_MIXED = 1
XRD_SF_DIRECT = 0
XRD_SF_RECURRENCE = 1
XRD_SF_AUTO = 2
XRD_NOALLOC_SCRATCH_BYTES = 64 << 20

_vp = C.c_void_p


class xrd_batch_desc(C.Structure):
    _fields_ = [
        ("n_crystals", C.c_int64), ("n_species", C.c_int32), ("precision", C.c_int32),
        ("lattice", _vp), ("atom_offset", _vp), ("two_theta_min", _vp), ("two_theta_max", _vp),
        ("wavelength", C.c_double), ("merge_tol", C.c_double), ("rel_threshold", C.c_double),
        ("friedel", C.c_int32), ("grid_capacity", C.c_int32),
        ("keep_sf_derivs", C.c_int32), ("sf_method", C.c_int32),
        ("frac", _vp), ("species", _vp), ("occ", _vp), ("bfac", _vp), ("sf_coeff", _vp),
        ("stream", _vp), ("forward_only", C.c_int32), ("sf_rpt", C.c_int32),
    ]


class xrd_sizes(C.Structure):
    _fields_ = [("n_crystals", C.c_int64), ("n_atoms", C.c_int64), ("refl_capacity", C.c_int64),
                ("peak_capacity", C.c_int64), ("workspace_bytes", C.c_int64), ("half_capacity", C.c_int64),
                ("noalloc_merge_bytes", C.c_int64)]


class xrd_refl(C.Structure):
    _fields_ = [("h", _vp), ("k", _vp), ("l", _vp), ("q", _vp), ("two_theta", _vp), ("lp", _vp),
                ("refl_offset", _vp)]


class xrd_peaks(C.Structure):
    _fields_ = [("two_theta", _vp), ("intensity", _vp), ("scaled", _vp), ("mult", _vp), ("first", _vp),
                ("perm", _vp), ("peak_offset", _vp)]


class xrd_line(C.Structure):
    _fields_ = [("peaks", C.POINTER(xrd_peaks)), ("q", _vp), ("weight", C.c_double)]


class xrd_line_peaks(C.Structure):
    _fields_ = [("two_theta", _vp), ("intensity", _vp), ("scaled", _vp), ("mult", _vp), ("d", _vp), ("line", _vp),
                ("source", _vp), ("peak_offset", _vp)]


class xrd_grid(C.Structure):
    _fields_ = [("t0", C.c_double), ("dt", C.c_double), ("n_points", C.c_int64), ("sigma", C.c_double),
                ("window_sigmas", C.c_double)]


class XrdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"xrd error {code}: {msg}")
        self.code = code


_lib = None

# name -> (argtypes, restype); the exported surface of include/xrd.h
SIGNATURES = {
    "xrd_batch_create": ([C.POINTER(xrd_batch_desc), C.POINTER(_vp)], C.c_int),
    "xrd_batch_sizes": ([_vp, C.POINTER(xrd_sizes)], C.c_int),
    "xrd_batch_upload": ([_vp, _vp], C.c_int),
    "xrd_batch_set_stream": ([_vp, _vp], C.c_int),
    "xrd_batch_set_lattice": ([_vp, _vp, _vp], C.c_int),
    "xrd_enumerate_hkl": ([_vp, _vp, C.POINTER(xrd_refl)], C.c_int),
    "xrd_structure_factors": ([_vp, _vp, C.POINTER(xrd_refl), _vp, _vp, _vp], C.c_int),
    "xrd_merge_peaks": ([_vp, _vp, C.POINTER(xrd_refl), _vp, C.POINTER(xrd_peaks)], C.c_int),
    "xrd_merge_peaks_noalloc": ([_vp, C.POINTER(xrd_refl), _vp, C.POINTER(xrd_peaks)], C.c_int),
    "xrd_pattern_forward": ([_vp, _vp, C.POINTER(xrd_refl), _vp, C.POINTER(xrd_grid), _vp], C.c_int),
    "xrd_pattern_backward": ([_vp, _vp, C.POINTER(xrd_refl), C.POINTER(xrd_grid), _vp, _vp, _vp, _vp], C.c_int),
    "xrd_autotune": ([_vp, _vp, C.POINTER(xrd_refl), C.POINTER(C.c_int32)], C.c_int),
    "xrd_batch_get_sf_rpt": ([_vp, C.POINTER(C.c_int32)], C.c_int),
    "xrd_combine_lines": ([C.c_int64, C.POINTER(xrd_line), C.POINTER(xrd_line), C.POINTER(xrd_line_peaks), _vp],
                          C.c_int),
    "xrd_preferred_orientation": ([_vp, _vp, C.POINTER(xrd_refl), _vp, _vp, _vp], C.c_int),
    "xrd_pattern_noise": ([_vp, C.c_int64, C.c_uint64, C.c_double, C.c_double, _vp], C.c_int),
    "xrd_peak_families": ([_vp, _vp, C.POINTER(xrd_refl), C.POINTER(xrd_peaks), C.c_int32, _vp, _vp, _vp, _vp],
                          C.c_int),
    "xrd_pattern_caglioti": ([_vp, _vp, C.POINTER(xrd_refl), _vp, C.POINTER(xrd_grid), C.c_double, C.c_double,
                              C.c_double, C.c_double, _vp], C.c_int),
    "xrd_read_counts": ([_vp, C.POINTER(xrd_refl), C.POINTER(xrd_peaks), _vp, _vp], C.c_int),
    "xrd_batch_destroy": ([_vp], None),
    "xrd_last_error": ([], C.c_char_p),
    "xrd_version": ([], C.c_char_p),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_11709_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(code: int):
    if code != XRD_OK:
        raise XrdError(code, lib().xrd_last_error().decode())
    return code


def xrd_batch_create(desc: xrd_batch_desc):
    h = _vp()
    check(lib().xrd_batch_create(C.byref(desc), C.byref(h)))
    return h


def xrd_batch_sizes(batch) -> xrd_sizes:
    s = xrd_sizes()
    check(lib().xrd_batch_sizes(batch, C.byref(s)))
    return s


def xrd_batch_set_lattice(batch, lattice_ptr: int, ws: int) -> int:
    """Status code (XRD_OK or XRD_ERR_CAPACITY when a search box would grow;
    other errors raise)."""
    code = lib().xrd_batch_set_lattice(batch, lattice_ptr, ws)
    if code not in (XRD_OK, XRD_ERR_CAPACITY):
        check(code)
    return code


def xrd_batch_set_stream(batch, stream: int):
    check(lib().xrd_batch_set_stream(batch, stream))


def xrd_batch_upload(batch, ws: int):
    check(lib().xrd_batch_upload(batch, ws))


def xrd_enumerate_hkl(batch, ws: int, refl: xrd_refl):
    check(lib().xrd_enumerate_hkl(batch, ws, C.byref(refl)))


def xrd_structure_factors(batch, ws: int, refl: xrd_refl, A: int, B: int, I: int):
    check(lib().xrd_structure_factors(batch, ws, C.byref(refl), A, B, I))


def xrd_merge_peaks(batch, ws: int, refl: xrd_refl, I: int, peaks: xrd_peaks):
    check(lib().xrd_merge_peaks(batch, ws, C.byref(refl), I, C.byref(peaks)))


def xrd_merge_peaks_noalloc(batch, refl: xrd_refl, I: int, peaks: xrd_peaks):
    check(lib().xrd_merge_peaks_noalloc(batch, C.byref(refl), I, C.byref(peaks)))


def xrd_pattern_forward(batch, ws: int, refl: xrd_refl, I: int, grid: xrd_grid, y: int):
    check(lib().xrd_pattern_forward(batch, ws, C.byref(refl), I, C.byref(grid), y))


def xrd_pattern_backward(batch, ws: int, refl: xrd_refl, grid: xrd_grid, dy: int, dfrac: int, dbfac: int,
                         dlat: int):
    check(lib().xrd_pattern_backward(batch, ws, C.byref(refl), C.byref(grid), dy, dfrac, dbfac, dlat))


def xrd_autotune(batch, ws: int, refl: xrd_refl):
    """Chosen (forward, adjoint) split thresholds, and the atom threshold of the
    recurrence under XRD_SF_AUTO (else -1)."""
    out = (C.c_int32 * 3)(0, 0, -1)
    check(lib().xrd_autotune(batch, ws, C.byref(refl), out))
    return int(out[0]), int(out[1]), int(out[2])


def xrd_batch_get_sf_rpt(batch) -> int:
    """The batch's tile shape of the direct structure-factor sums (reflections per lane)."""
    out = C.c_int32(0)
    check(lib().xrd_batch_get_sf_rpt(batch, C.byref(out)))
    return int(out.value)


def xrd_combine_lines(n_crystals: int, line0: xrd_line, line1, out: xrd_line_peaks, stream: int):
    """line1 None: line0 alone."""
    check(lib().xrd_combine_lines(n_crystals, C.byref(line0), C.byref(line1) if line1 is not None else None,
                                  C.byref(out), stream))


def xrd_preferred_orientation(batch, ws: int, refl: xrd_refl, hp: int, march_r: int, I: int):
    check(lib().xrd_preferred_orientation(batch, ws, C.byref(refl), hp, march_r, I))


def xrd_peak_families(batch, ws: int, refl: xrd_refl, peaks: xrd_peaks, rule: int, n_families: int,
                      family_of: int, family_label: int, family_mult: int):
    check(lib().xrd_peak_families(batch, ws, C.byref(refl), C.byref(peaks), int(rule), n_families, family_of,
                                  family_label, family_mult))


def xrd_pattern_caglioti(batch, ws: int, refl: xrd_refl, I: int, grid: xrd_grid, U: float, V: float, W: float,
                         y: int, eta: float = 0.0):
    check(lib().xrd_pattern_caglioti(batch, ws, C.byref(refl), I, C.byref(grid), float(U), float(V), float(W),
                                     float(eta), y))


def xrd_pattern_noise(batch, n_points: int, seed: int, rel: float, abs_: float, y: int):
    check(lib().xrd_pattern_noise(batch, int(n_points), int(seed) & (2**64 - 1), float(rel), float(abs_), y))


def xrd_read_counts(batch, refl, peaks, host_refl_offset, host_peak_offset):
    check(lib().xrd_read_counts(batch, C.byref(refl) if refl is not None else None,
                                C.byref(peaks) if peaks is not None else None,
                                host_refl_offset, host_peak_offset))


def xrd_batch_destroy(batch):
    if batch:
        lib().xrd_batch_destroy(batch)


def xrd_last_error() -> str:
    return lib().xrd_last_error().decode()


def xrd_version() -> str:
    return lib().xrd_version().decode()
