#!/usr/bin/env python3
"""Benchmark of the powder-XRD hot path on one MI355X.

Workload: the uneven batch of 1024 synthetic triclinic crystals (a, b, c ~
U(3, 15) A, angles U(60, 120) deg, 1-200 atoms log-uniform, 1-10 species
per crystal, Cu K-alpha, 2theta 10-90 deg, merge tolerance 1e-5 deg), seed 1.

One step = the whole hot path over that batch, inputs resident in HBM:
reciprocal-lattice enumeration with q, 2theta and LP; structure factors and
intensities; sort, anchor-rule merge and 0-100 scaling; the Gaussian-
broadened pattern (4001 points over 10-90 deg, sigma 0.1 deg); and the
adjoint of that pattern for a fixed synthetic dL/dy (gradients with respect
to fractional coordinates, B factors and lattice parameters).  The step runs
either as eager launches on one stream or captured once into a HIP graph and
replayed; a timed region holds exactly ``--steps`` steps between two device
synchronisations.  By default both launch modes are timed, each over its own
``--steps`` steps, and the faster is the headline (the step is not
launch-bound: the host enqueues its dozen kernels well within the device
time, and each graph replay adds a few microseconds at its boundary).

Printed: one JSON line (value = patterns per second of the mixed-precision
path), with the double-precision path timed the same way (every reflection,
and Friedel-halved like the mixed path), the structure-factor kernel's
roofline and those of the other long kernels of the step, the oracle timed on
the host as a CPU baseline, and, under ``configs``, the other workloads: the
rock-salt cell, the 16 large cells (2000-5000 atoms) and the 256-crystal
differentiation workload, each with its own oracle timing.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "structure-factor terms/s & patterns/s, FP32-mixed vs FP64 at ≤1e-4 rel err"
GRID = dict(t0=10.0, dt=0.02, n_points=4001, sigma=0.1, window_sigmas=8.0)
CLOCK_HZ = 2.4e9
N_CU = 256
# Peak lane-operations per compute unit and clock on gfx950, one set of rates
# for every ALU roofline below: FP64 78.6 TFLOP/s = 64 FMA lanes, FP32 157.3
# TFLOP/s = 128 FMA lanes (the published figure counts packed FP32; this
# library is built without packed FP32, so the figure is a conservative
# ceiling), transcendentals (v_sin/v_cos/v_exp_f32) at half the unpacked FP32
# lane rate, 32.  The instruction-rate microbenchmark (xrd_rates) measures
# 51 / 87 / 28-29 of these on the box, and the structure-factor term mix at
# 2.31e12 terms/s (profiles/rates_gfx950.md); an instruction mix costs the sum
# of its classes' shares (the microbenchmark's term mix runs within 2% of
# that sum).
RATE_F32, RATE_F64, RATE_TRANS = 128.0, 64.0, 32.0
# Algorithmic work per unit of each ALU-bound kernel (ops by class):
UNIT_OPS = {
    # k_sf, mixed, keeping dF/ds^2: per structure-factor term, the phase
    # h.x (3 FP64), reduction mod 1 and conversion (2 FP64-rate), sin + cos +
    # the weight's exp2 (3 transcendental), the weight exponent and two
    # multiply-adds for F, one product and two multiply-adds for dF/ds^2 (6 FP32)
    "k_sf": dict(f64=5, trans=3, f32=6),
    # k_sf_bw, mixed, atom-gradient pass of the crystals up to 512 atoms: per
    # term the same phase and weight (5 FP64-rate, 3 transcendental, 1 FP32),
    # P = w (gB cos - gA sin) and Q = w (gA cos + gB sin) (6 FP32) and the
    # four sums h P, k P, l P, s^2 Q (4 FP32)
    "k_sf_bw": dict(f64=5, trans=3, f32=11),
    # k_broaden_gather, mixed: per (grid point, reflection in its window)
    # pair, the offset x - 2theta, the window test and the conversion (3
    # FP64-rate), one exp2 (1 transcendental), the square, the scale and the
    # weighted sum (3 FP32)
    "k_broaden_gather": dict(f64=3, trans=1, f32=3),
}


def progress(msg):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def unit_peak_per_s(kernel):
    """Units per second at the peak rates (costs of the classes added)."""
    ops = UNIT_OPS[kernel]
    clk = ops["f64"] / RATE_F64 + ops["trans"] / RATE_TRANS + ops["f32"] / RATE_F32
    return N_CU * CLOCK_HZ / clk


def term_peak_per_s():
    return unit_peak_per_s("k_sf")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--launch", choices=["auto", "graph", "eager"], default="auto",
                    help="launch mode of the timed steps (auto: time both, report the faster)")
    ap.add_argument("--no-graph", action="store_true", help="same as --launch eager")
    ap.add_argument("--no-fp64", action="store_true", help="skip the double-precision comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default structure-factor split thresholds")
    ap.add_argument("--no-doublet", action="store_true", help="skip the Cu K-alpha doublet forward timing")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the rock-salt, large-cell and gradient workloads (headline workload only)")
    ap.add_argument("--no-rates", action="store_true", help="skip the instruction-rate microbenchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters), then exit")
    ap.add_argument("--config", choices=["rocksalt", "large_cells", "gradient_256", "database_stream"],
                    help="only run this workload's leg (printed as one JSON object), then exit")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 28  # 2^28 float32 = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


class Pipeline:
    """Buffers and the step of one precision, on a stream of its own."""

    def __init__(self, batch, precision, dy_seed=7, friedel=None):
        import torch
        from paper_2602_11709_amd.api import Grid, XrdBatch
        self.torch = torch
        self.grid = Grid(**GRID)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            t0 = time.perf_counter()
            # the step differentiates the pattern: the forward keeps dF/ds^2
            self.xb = XrdBatch(batch, precision=precision, friedel=friedel, keep_sf_derivs=True)
            self.plan_ms = (time.perf_counter() - t0) * 1e3
            xb = self.xb
            self.refl = xb.new_reflections()
            self.sf = xb.new_sf()
            self.pk = xb.new_peaks()
            self.y = torch.empty(batch.n_crystals, self.grid.n_points, dtype=torch.float64, device="cuda")
            g = torch.Generator(device="cpu").manual_seed(dy_seed)
            self.dy = torch.randn(batch.n_crystals, self.grid.n_points, generator=g,
                                  dtype=torch.float64).cuda()
            self.grads = xb.new_grads()
        self.graph = None

    # stages of one step
    def enumerate(self):
        self.xb.enumerate(self.refl)

    def structure_factors(self):
        self.xb.structure_factors(self.refl, self.sf)

    def merge(self):
        self.xb.merge(self.refl, self.sf[2], self.pk)

    def pattern(self):
        self.xb.pattern_forward(self.refl, self.sf[2], self.grid, self.y)

    def adjoint(self):
        self.xb.pattern_backward(self.refl, self.grid, self.dy, self.grads)

    def step(self):
        self.enumerate()
        self.structure_factors()
        self.merge()
        self.pattern()
        self.adjoint()

    def outputs(self):
        n = int(self.refl.refl_offset[-1])
        m = int(self.pk.peak_offset[-1])
        return {"I": self.sf[2][:n].clone(), "pk_i": self.pk.intensity[:m].clone(),
                "pk_tt": self.pk.two_theta[:m].clone(), "mult": self.pk.mult[:m].clone(),
                "y": self.y.clone(), "dfrac": self.grads[0].clone(), "dlat": self.grads[2].clone()}

    def capture(self):
        torch = self.torch
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.step()

    def run(self, graph):
        if graph:
            self.graph.replay()
        else:
            with self.torch.cuda.stream(self.stream):
                self.step()

    def time_call(self, fn, reps, trials=3):
        """Average device time of ``fn`` over ``reps`` back-to-back calls (events on
        the batch stream), the best of ``trials`` such runs: a stall of the
        launching host thread leaves the device idle between calls and would
        count as device time."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        with torch.cuda.stream(self.stream):
            fn()
            for _ in range(trials):
                e0.record(self.stream)
                for _ in range(reps):
                    fn()
                e1.record(self.stream)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) / reps)
        return best


class Forward:
    """Enumerate, structure factors and merge (the forward pattern of the
    paper's calculator) of one batch and precision, captured in a HIP graph
    on a stream of its own."""

    def __init__(self, batch, precision, friedel=None, sf_method="direct", autotune=False):
        import torch
        from paper_2602_11709_amd.api import XrdBatch
        self.torch = torch
        self.batch = batch
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.xb = XrdBatch(batch, precision=precision, friedel=friedel, sf_method=sf_method, forward_only=True)
            self.refl = self.xb.new_reflections()
            self.sf = self.xb.new_sf()
            self.pk = self.xb.new_peaks()
            self.tuned = None
            if autotune:
                # set-up: tile shape and split-K of the forward sums on the enumerated reflections
                self.xb.enumerate(self.refl)
                fwd, _, rec = self.xb.autotune(self.refl)
                self.tuned = {"reflections_per_lane": self.xb.sf_rpt, "split_atoms": fwd,
                              "recurrence_min_atoms": rec if rec >= 0 else None}
            self.step()
        torch.cuda.synchronize()
        self.n_refl = int(self.refl.refl_offset[-1])
        self.n_peaks = int(self.pk.peak_offset[-1])
        eager = self.snapshot()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.step()
        self.graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, self.snapshot()):
            if not torch.equal(a, b):
                raise RuntimeError("graph replay differs from eager")

    def structure_factors(self):
        self.xb.structure_factors(self.refl, self.sf)

    def step(self):
        self.xb.enumerate(self.refl)
        self.structure_factors()
        self.xb.merge(self.refl, self.sf[2], self.pk)

    def snapshot(self):
        return [self.sf[2][:self.n_refl].clone(), self.pk.intensity[:self.n_peaks].clone(),
                self.pk.mult[:self.n_peaks].clone()]

    def replay_ms(self, steps):
        torch = self.torch
        self.graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.graph.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def sf_ms(self, reps):
        return time_on_stream(self.torch, self.stream, self.structure_factors, reps)

    def terms(self):
        """(all terms sum_c R_c N_c, evaluated terms: one reflection of each
        Friedel pair when the batch pairs them)."""
        ro = self.refl.refl_offset.cpu().numpy()
        full = int((np.diff(ro) * np.diff(self.batch.atom_offset)).sum())
        return full, full // 2 if self.xb.friedel else full

    def peaks(self):
        po = self.pk.peak_offset.cpu().numpy()
        return po, self.pk.intensity[:self.n_peaks].double().cpu().numpy(), self.pk.mult[:self.n_peaks].cpu().numpy()


def time_on_stream(torch, stream, fn, reps, trials=3):
    """Average device time of ``fn`` over ``reps`` back-to-back calls (HIP
    events on ``stream``, where the library enqueues its work), best of
    ``trials``."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    with torch.cuda.stream(stream):
        fn()
        for _ in range(trials):
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / reps)
    return best


def strong_peak_rel_err(po, got, ref):
    """Largest relative error of ``got`` against ``ref`` over the peaks with
    at least 1e-3 of their crystal's strongest peak."""
    worst = 0.0
    for c in range(len(po) - 1):
        s = slice(po[c], po[c + 1])
        if s.stop > s.start and ref[s].max() > 0:
            strong = ref[s] >= 1e-3 * ref[s].max()
            worst = max(worst, float(np.max(np.abs(got[s][strong] - ref[s][strong]) / ref[s][strong])))
    return worst


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def host_threads():
    """Oracle threads: the host cores this process may use, at most 16 (one
    GPU's share of the host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def leg_recurrence(batch, reps):
    """Structure factors by the row recurrence against the direct sum on one
    workload, both precisions (Friedel-halved, so both evaluate the same
    reflections): device time of the structure-factor call (the recurrence's
    includes building its segments), evaluated terms per second, the
    recurrence kernel's own time, and the forward step (enumerate, structure
    factors, merge) per replay."""
    progress("leg_recurrence")
    import torch
    out = {}
    for precision in ("mixed", "fp64"):
        r = {}
        for method in ("direct", "recurrence"):
            f = Forward(batch, precision, True, sf_method=method)
            ms = f.sf_ms(reps)
            _, ev = f.terms()
            r[method] = {"sf_call_ms": round(ms, 5), "sf_terms_per_s": round(ev / (ms * 1e-3), 1),
                         "forward_ms": round(f.replay_ms(5), 5)}
            if method == "recurrence":
                kus = kernel_device_us(torch, f.stream, f.structure_factors, 3, ["k_sf_rec<", "k_seg_"])
                r[method]["kernel_us"] = {k.rstrip("<_"): round(v, 2) for k, v in kus.items()}
            del f
        r["speedup_sf_call"] = round(r["direct"]["sf_call_ms"] / r["recurrence"]["sf_call_ms"], 3)
        out[precision] = r
    return out


def leg_database(chunk=4096, planners=6):
    """The database-scale stream: 100 000 synthetic crystals shaped like the
    structure databases of the paper's benchmarks (Mo K-alpha, 2theta 2-60),
    forward patterns (enumerate, structure factors, merge, scaled peaks) in
    chunks planned on host threads while the GPU computes; peaks stay on the
    device.  Also per bin of reflection count (the paper's Fig. 8 bins), the
    bins' crystals streamed on their own.  Chunks of 4096 crystals: with 8192
    the launch tables' upload (pageable host memory, about 3.6 ms a chunk
    against 0.4 ms at 4096) holds the GPU up."""
    progress("leg_database")
    import oracle
    from paper_2602_11709_amd import synth
    from paper_2602_11709_amd.stream import DatabaseStream
    t0 = time.perf_counter()
    b = synth.database_stream()
    gen_s = time.perf_counter() - t0
    out = {"workload": "database_stream: 100000 crystals, atoms log-normal (median 20, sigma_log 1, 1-1000), "
                       "lengths 2.6 A N^(1/3) U(0.8,1.2), angles U(60,120), Mo 0.71073 A, 2theta 2-60, seed 3",
           "chunk": chunk, "planners": planners, "generate_s": round(gen_s, 2)}
    counts = np.zeros(b.n_crystals, np.int64)

    def keep_counts(cp):
        counts[cp.first:cp.first + cp.n_crystals] = np.diff(cp.refl_offset)

    for precision in ("mixed", "fp64"):
        # untimed warm-up (first allocations and launches) on the first crystals
        DatabaseStream(b.subset(range(2 * chunk)), chunk=chunk, precision=precision, planners=planners).run()
        st = DatabaseStream(b, chunk=chunk, precision=precision, planners=planners).run(
            keep_counts if precision == "mixed" else None)
        out[precision] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
    bins = {}
    for lo, hi, name in ((0, 10, "<=10"), (10, 100, "10-100"), (100, 100000, "100-1e5"), (100000, None, ">1e5")):
        idx = np.nonzero((counts > lo) & ((counts <= hi) if hi is not None else True))[0]
        if lo == 0:
            idx = np.nonzero(counts <= 10)[0]
        entry = {"crystals": int(len(idx)), "reflections": int(counts[idx].sum())}
        if len(idx):
            st = DatabaseStream(b.subset(idx), chunk=chunk, planners=planners).run()
            entry.update(patterns_per_s=round(st["patterns_per_s"], 1),
                         patterns_per_s_device=round(st["patterns_per_s_device"], 1), wall_s=round(st["wall_s"], 4))
        bins[name] = entry
    out["bins_mixed"] = bins
    # oracle: the first 2000 crystals on the host threads
    threads = host_threads()
    sub = b.subset(range(2000))
    t0 = time.perf_counter()
    oracle.pattern_batch(sub, threads=threads, keep=False)
    wall = time.perf_counter() - t0
    out["cpu_oracle"] = {"patterns_per_s": round(2000 / wall, 1), "threads": threads,
                         "wall_s_100000_extrapolated": round(wall * 50, 1),
                         "sample": f"oracle forward patterns of the first 2000 crystals on {threads} threads, "
                                   f"{wall:.2f} s; the whole stream extrapolated x50"}
    return out


def leg_rocksalt(steps):
    """The single rock-salt cell (the closed-form pin case), plain FP64 path
    as the configuration names it, and the mixed path: forward pattern."""
    progress("leg_rocksalt")
    import oracle
    from paper_2602_11709_amd import synth
    b = synth.rocksalt()
    out = {"workload": "rocksalt: 1 cubic cell a = 5.64 A, 8 atoms, Cu 1.54184 A, 2theta 0-90, tol 1e-5"}
    for precision in ("fp64", "mixed"):
        f = Forward(b, precision)
        ms = f.replay_ms(steps)
        sf = f.sf_ms(50)
        full, ev = f.terms()
        out[precision] = {"ms_per_pattern": round(ms, 5), "patterns_per_s": round(1e3 / ms, 1),
                          "sf_kernel_ms": round(sf, 5), "sf_terms_per_s": round(ev / (sf * 1e-3), 1),
                          "reflections": f.n_refl, "peaks": f.n_peaks}
    n, t0 = 0, time.perf_counter()
    while n == 0 or time.perf_counter() - t0 < 1.0:
        oracle.pattern(b, 0)
        n += 1
    wall = time.perf_counter() - t0
    out["cpu_oracle"] = {"patterns_per_s": round(n / wall, 1), "threads": 1,
                         "sample": f"{n} forward patterns of the cell, one thread"}
    return out


def oracle_sf_rate(batch, crystals, n_sample, threads, seed=0):
    """Oracle structure-factor terms per second on a random sample of
    ``n_sample`` reflections of each listed crystal, split over ``threads``
    host threads (the oracle's C routine runs without the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    rng = np.random.default_rng(seed)
    jobs = []
    for c in crystals:
        hkl, q, _, _ = oracle.enumerate_hkl(batch.lattice[c], batch.wavelength, float(batch.two_theta_min[c]),
                                            float(batch.two_theta_max[c]))
        pick = rng.choice(len(q), size=min(n_sample, len(q)), replace=False)
        sl = batch.atoms_of(c)
        args = (batch.frac[sl], batch.species[sl], batch.occ[sl], batch.bfac[sl], batch.sf_coeff)
        for part in np.array_split(pick, threads):
            jobs.append((hkl[part], q[part], args))
    terms = sum(len(j[1]) * len(j[2][1]) for j in jobs)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda j: oracle.structure_factors(j[0], j[1], *j[2]), jobs))
    return terms / (time.perf_counter() - t0), terms


def leg_large_cells(steps):
    """The large-cell stress batch (16 cells of 2000-5000 atoms, ~2e5-5e5
    reflections each): mixed path, plain FP64 path evaluating every
    reflection, and FP64 with Friedel halving (so the precision alone is
    compared with the mixed path).  The structure-factor method is the
    library's "auto" choice, which the autotuner settles per batch (direct
    sums or the row recurrence above an atom threshold)."""
    from paper_2602_11709_amd import synth
    b = synth.large_cells()
    out = {"workload": "large_cells: 16 cells (8 monoclinic, 8 triclinic), a,b,c~U(30,50) A, 2000-5000 atoms, "
                       "20 species, occ U(0.5,1), Cu 1.54184 A, 2theta 5-120, seed 2"}
    peaks = {}
    for name, precision, friedel in (("mixed", "mixed", True), ("fp64", "fp64", False),
                                     ("fp64_friedel", "fp64", True)):
        progress(f"large cells, {name}")
        f = Forward(b, precision, friedel, sf_method="auto", autotune=True)
        ms = f.replay_ms(steps)
        sf = f.sf_ms(3)
        full, ev = f.terms()
        out[name] = {"ms_per_step": round(ms, 4), "patterns_per_s": round(b.n_crystals / (ms * 1e-3), 2),
                     "sf_kernel_ms": round(sf, 4), "sf_terms_per_s": round(ev / (sf * 1e-3), 1),
                     "sf_terms_per_s_effective": round(full / (sf * 1e-3), 1), "evaluated_terms": ev,
                     "reflections": f.n_refl, "peaks": f.n_peaks, "autotune": f.tuned}
        peaks[name] = f.peaks()
        del f
    # one cell alone (the paper times single large structures): the median
    # cell by atom count, its whole forward as one graph replay
    na = np.diff(b.atom_offset)
    med = int(np.argsort(na)[len(na) // 2])
    progress("large cells, one cell")
    f = Forward(b.subset([med]), "mixed", True, sf_method="auto", autotune=True)
    ms = f.replay_ms(10)
    out["one_cell"] = {"crystal": med, "atoms": int(na[med]), "reflections": f.n_refl, "peaks": f.n_peaks,
                       "ms_per_pattern": round(ms, 4), "precision": "mixed",
                       "note": "enumerate, structure factors, merge of one cell, graph replay"}
    del f
    po, got, m1 = peaks["mixed"]
    _, ref, m2 = peaks["fp64"]
    out["mixed_vs_fp64_same_peaks"] = bool(np.array_equal(m1, m2))
    out["mixed_vs_fp64_max_rel_err_strong_peaks"] = strong_peak_rel_err(po, got, ref) if np.array_equal(m1, m2) else None
    out["speedup_mixed_vs_fp64_friedel_sf_kernel"] = round(out["fp64_friedel"]["sf_kernel_ms"] / out["mixed"]["sf_kernel_ms"], 3)
    # oracle: structure factors of a reflection sample of a monoclinic and a triclinic cell
    threads = host_threads()
    rate1, t1 = oracle_sf_rate(b, [0, 8], 600, 1)
    rate_n, tn = oracle_sf_rate(b, [0, 8], 600 * threads, threads, seed=1)
    per_crystal = out["fp64"]["evaluated_terms"] / b.n_crystals
    out["cpu_oracle"] = {"sf_terms_per_s_1_thread": round(rate1, 1), "sf_terms_per_s": round(rate_n, 1),
                         "threads": threads, "patterns_per_s_extrapolated": round(rate_n / per_crystal, 4),
                         "sample": f"oracle structure factors of random reflections of crystals 0 (monoclinic) "
                                   f"and 8 (triclinic): {t1} terms on 1 thread, {tn} on {threads}; patterns/s "
                                   f"extrapolated from terms/s and the batch's mean {per_crystal:.3g} terms per "
                                   f"crystal (every reflection, as the oracle evaluates them)"}
    return out


def leg_gradients(steps):
    """The differentiation workload (256 crystals of 50-500 atoms, 4001-point
    pattern): one step = enumerate, structure factors keeping dF/ds^2, the
    broadened pattern and its adjoint for a fixed dL/dy, mixed and FP64."""
    progress("leg_gradients")
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import torch
    from paper_2602_11709_amd import synth
    from paper_2602_11709_amd.api import Grid, XrdBatch
    gp = synth.gradient_problem()
    b = gp.batch
    grid = Grid(gp.grid_t0, gp.grid_dt, gp.grid_n, gp.sigma, gp.window_sigmas)
    out = {"workload": "gradient_problem: 256 crystals of 50-500 atoms (database lattice rule), Cu 1.54184 A, "
                       "enumerated over 9.2-90.8 deg, 4001-point grid 10-90 deg, sigma 0.1 deg, seed 4; step = "
                       "enumerate + structure factors + pattern + adjoint (dL/dfrac, dL/dlattice, dL/dB)"}
    for precision in ("mixed", "fp64"):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            xb = XrdBatch(b, precision=precision, grid_capacity=grid.n_points, keep_sf_derivs=True)
            refl, sf = xb.new_reflections(), xb.new_sf()
            y = torch.empty(b.n_crystals, grid.n_points, dtype=torch.float64, device="cuda")
            dy = torch.randn(b.n_crystals, grid.n_points, generator=torch.Generator().manual_seed(5),
                             dtype=torch.float64).cuda()
            grads = xb.new_grads()
            # set-up: tile shape and split-K of both sums tuned on the enumerated reflections
            xb.enumerate(refl)
            split_fwd, split_bw, _ = xb.autotune(refl)
            tuned = {"reflections_per_lane": xb.sf_rpt, "split_atoms_forward": split_fwd,
                     "split_atoms_adjoint": split_bw}

        def fwd():
            xb.enumerate(refl)
            xb.structure_factors(refl, sf)
            xb.pattern_forward(refl, sf[2], grid, y)

        def step():
            fwd()
            xb.pattern_backward(refl, grid, dy, grads)

        with torch.cuda.stream(s):
            step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        fwd_ms = time_on_stream(torch, s, fwd, 5)
        bwd_ms = time_on_stream(torch, s, lambda: xb.pattern_backward(refl, grid, dy, grads), 5)
        n_refl = np.diff(refl.refl_offset.cpu().numpy())
        full = int((n_refl * b.counts()).sum())
        out[precision] = {"ms_per_step": round(ms, 4), "patterns_per_s": round(b.n_crystals / (ms * 1e-3), 1),
                          "forward_ms": round(fwd_ms, 4), "adjoint_ms": round(bwd_ms, 4), "autotune": tuned,
                          "reflections": int(n_refl.sum()), "sf_terms": full}
        del g, xb
    # the autograd path as an optimisation loop calls it: plan, forward, backward
    from paper_2602_11709_amd.api import xrd_pattern
    frac = torch.tensor(b.frac, device="cuda", requires_grad=True)
    lat = torch.tensor(b.lattice, requires_grad=True)
    bf = torch.tensor(b.bfac, device="cuda", requires_grad=True)
    times = []
    for _ in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        yy = xrd_pattern(frac, lat, bf, b, grid, precision="mixed")
        yy.backward(torch.ones_like(yy))
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    out["autograd_iteration_ms"] = {"first": round(times[0], 2), "later_best": round(min(times[1:]), 2)}
    # oracle: forward broadened patterns of a crystal sample (it has no adjoint)
    threads = host_threads()
    ga = (gp.grid_t0, gp.grid_dt, gp.grid_n, gp.sigma, gp.window_sigmas)
    t0 = time.perf_counter()
    for c in range(4):
        oracle.broadened(b, c, *ga)
    one = 4 / (time.perf_counter() - t0)
    n = 4 * threads
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda c: oracle.broadened(b, c, *ga), range(n)))
    alln = n / (time.perf_counter() - t0)
    out["cpu_oracle"] = {"patterns_per_s_1_thread": round(one, 2), "patterns_per_s": round(alln, 2),
                         "threads": threads, "sample": f"forward broadened patterns (enumerate, structure "
                         f"factors, LP, broadening; the oracle has no adjoint) of crystals 0-3 on 1 thread and "
                         f"0-{n - 1} on {threads}"}
    return out


def rates_live():
    """The instruction-rate microbenchmark, run once as a child program."""
    import subprocess
    exe = os.path.join(HERE, "paper_2602_11709_amd", "xrd_rates")
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
        return json.loads(r.stdout) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError):
        return None


def frontend_rate(batch, n=128):
    """The calculator front-end (get_patterns, Cu K-alpha1 + K-alpha2, families
    by indices) on the workload's first n crystals: whole calls, wall time,
    including planning both lines, the device work, the lines' combination on
    the device and the host's per-peak hkl lists (Python objects); best of 3."""
    import time as _t
    import torch
    from paper_2602_11709_amd import frontend
    sub = batch.subset(range(min(n, batch.n_crystals)))
    best, peaks = float("inf"), 0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        pats = frontend.get_patterns(sub, "CuKa12")
        best = min(best, _t.perf_counter() - t0)
        peaks = sum(len(p.x) for p in pats)
    return {"crystals": sub.n_crystals, "peaks": peaks, "s": round(best, 4),
            "patterns_per_s": round(sub.n_crystals / best, 1), "peaks_per_s": round(peaks / best, 1),
            "call": "frontend.get_patterns(first crystals of the workload, 'CuKa12'): wall time of whole calls"}


def doublet_ms(batch, reps=20):
    """Forward patterns (peaks and the broadened pattern) of the workload under
    Cu K-alpha1 and K-alpha2 (two lines of the calculator front-end): both
    lines' enumerate, structure factors, merge and pattern captured in one
    graph; average replay time in ms."""
    import dataclasses
    import torch
    from paper_2602_11709_amd import frontend
    from paper_2602_11709_amd.api import Grid, XrdBatch
    grid = Grid(**GRID)
    s = torch.cuda.Stream()
    parts = []
    with torch.cuda.stream(s):
        for lam, _, _ in frontend.lines_of("CuKa12"):
            xb = XrdBatch(dataclasses.replace(batch, wavelength=lam), precision="mixed")
            parts.append((xb, xb.new_reflections(), xb.new_sf(), xb.new_peaks(),
                          torch.empty(batch.n_crystals, grid.n_points, dtype=torch.float64, device="cuda")))

    def step():
        for xb, refl, sf, pk, y in parts:
            xb.enumerate(refl)
            xb.structure_factors(refl, sf)
            xb.merge(refl, sf[2], pk)
            xb.pattern_forward(refl, sf[2], grid, y)

    with torch.cuda.stream(s):
        step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def augment_ms(p: Pipeline):
    """Device time of the ML augmentations on the workload's reflections and
    patterns (after every other measurement: they change the buffers)."""
    import torch
    from paper_2602_11709_amd import capi
    n_c = p.xb.n_crystals
    g = torch.Generator().manual_seed(11)
    hp = torch.randn(n_c, 3, generator=g, dtype=torch.float64).cuda()
    mr = (0.5 + torch.rand(n_c, generator=g, dtype=torch.float64)).cuda()
    torch.cuda.synchronize()
    po = p.time_call(lambda: capi.xrd_preferred_orientation(p.xb.handle, p.xb.ws, p.refl.c(), hp.data_ptr(),
                                                            mr.data_ptr(), p.sf[2].data_ptr()), 20)
    nz = p.time_call(lambda: capi.xrd_pattern_noise(p.xb.handle, p.y.shape[1], 12345, 0.05, 0.01,
                                                    p.y.data_ptr()), 20)
    # Caglioti widths of a laboratory diffractometer (FWHM 0.06-0.2 degrees over the range)
    cg = p.time_call(lambda: capi.xrd_pattern_caglioti(p.xb.handle, p.xb.ws, p.refl.c(), p.sf[2].data_ptr(),
                                                       p.grid.c(), 0.02, -0.005, 0.004, p.y.data_ptr()), 20)
    pv = p.time_call(lambda: capi.xrd_pattern_caglioti(p.xb.handle, p.xb.ws, p.refl.c(), p.sf[2].data_ptr(),
                                                       p.grid.c(), 0.02, -0.005, 0.004, p.y.data_ptr(), 0.5), 20)
    return {"preferred_orientation_ms": round(po, 5), "noise_ms": round(nz, 5),
            "caglioti_pattern_ms": round(cg, 5), "pseudo_voigt_pattern_ms": round(pv, 5), "noise_points": int(p.y.numel())}


def families_ms(p: Pipeline):
    """Device time of the grouping of equivalent reflections over every merged
    peak of the workload, per rule (outputs preallocated)."""
    import torch
    from paper_2602_11709_amd import capi
    rc = max(p.xb.refl_capacity, 1)
    dev = "cuda"
    out = (torch.empty(rc, dtype=torch.int32, device=dev), torch.empty(rc, dtype=torch.int32, device=dev),
           torch.empty(rc, dtype=torch.int64, device=dev), torch.empty(rc, dtype=torch.int32, device=dev))
    ptrs = [t.data_ptr() for t in out]
    res = {}
    for name, rule in (("indices", 0), ("lattice", 1)):
        res[name + "_ms"] = round(p.time_call(lambda: capi.xrd_peak_families(p.xb.handle, p.xb.ws, p.refl.c(),
                                                                             p.pk.c(), rule, *ptrs), 20), 5)
    return res


def timed(p: Pipeline, steps, warmup, graph):
    torch = p.torch
    for _ in range(warmup):
        p.run(graph)
    torch.cuda.synchronize()  # barrier of the single rank
    t0 = time.perf_counter()
    for _ in range(steps):
        p.run(graph)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def workload_stats(batch, refl_offset):
    counts = np.diff(batch.atom_offset)
    refl = np.diff(refl_offset)
    return int(refl.sum()), int((refl * counts).sum())


TRAFFIC_SOURCES = ("sf.hip", "api.cpp")  # the kernel, and the host code that orders its work


def sources_sha256():
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(HERE, "paper_2602_11709_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_record():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, valid only while the kernel source and its work ordering are
    unchanged."""
    path = os.path.join(HERE, "profiles", "sf_mixed_triclinic_1024_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != sources_sha256():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(batch):
    """The oracle on the host: whole passes over the workload on the host
    threads until about 20 thread-seconds, and one thread on a crystal
    sample for the single-core figure."""
    progress("cpu_baseline")
    import oracle
    threads = host_threads()
    model, visible = cpu_info()
    passes, wall = 0, 0.0
    t0 = time.perf_counter()
    while passes < 64 and (passes == 0 or wall * threads < 20.0):
        oracle.pattern_batch(batch, threads=threads, keep=False)
        passes += 1
        wall = time.perf_counter() - t0
    # one thread: every 8th crystal (128 of them, the workload's size mix)
    sub = batch.subset(range(0, batch.n_crystals, 8))
    t0 = time.perf_counter()
    oracle.pattern_batch(sub, threads=1, keep=False)
    one = sub.n_crystals / (time.perf_counter() - t0)
    return {"value": passes * batch.n_crystals / wall, "unit": "patterns/s", "cores": threads, "kind": "oracle",
            "single_thread_value": round(one, 1), "host_cores_visible": visible, "cpu_model": model,
            "sample": f"{passes} passes over all {batch.n_crystals} crystals of the workload, forward pattern "
                      f"only (enumerate, structure factors, LP, sort, merge, scale; the oracle has no "
                      f"adjoint), plain FP64 C on {threads} OpenMP threads (of {visible} visible), "
                      f"{wall:.2f} s wall (~{wall * threads:.0f} thread-seconds); single_thread_value: every "
                      f"8th crystal ({sub.n_crystals}) on one thread"}


def entry_window_pairs(p):
    """(grid point, reflection) pairs the broadened pattern sums: for each
    evaluated reflection (one of each Friedel pair when the batch pairs
    them), the grid points within window_sigmas * sigma of its 2theta."""
    g = p.grid
    ro = p.refl.refl_offset.cpu().numpy()
    tt = p.refl.two_theta[: int(ro[-1])].cpu().numpy()
    if p.xb.friedel:
        keep = np.concatenate([np.arange((a + b) // 2, b) for a, b in zip(ro[:-1], ro[1:])])
        tt = tt[keep]
    half = g.window_sigmas * g.sigma
    lo = np.maximum(np.ceil((tt - half - g.t0) / g.dt), 0)
    hi = np.minimum(np.floor((tt + half - g.t0) / g.dt), g.n_points - 1)
    return int(np.maximum(hi - lo + 1, 0).sum())


def kernel_device_us(torch, stream, fn, reps, names):
    """Average device time (us) per launch of the named kernels over ``reps``
    eager calls of ``fn`` on ``stream``, from the profiler's kernel records
    (kernels launched by the library included)."""
    from torch.profiler import ProfilerActivity, profile
    with torch.cuda.stream(stream):
        fn()
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        with torch.cuda.stream(stream):
            for _ in range(reps):
                fn()
        torch.cuda.synchronize()
    out = {}
    for e in prof.key_averages():
        for n in names:
            if n in e.key and e.count:
                out[n] = out.get(n, 0.0) + e.device_time_total / e.count
    return out


def alu_roofline(kernel, units, us, unit_name, note):
    peak = unit_peak_per_s(kernel)
    achieved = units / (us * 1e-6)
    return {"kernel": kernel, "bound": "alu", "achieved": round(achieved / 1e9, 3), "peak": round(peak / 1e9, 3),
            "unit": f"G{unit_name}/s", "frac": round(achieved / peak, 4), "per_launch_units": units,
            "avg_launch_us": round(us, 2), "ops_per_unit": UNIT_OPS[kernel], "timing": note}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the batch would shard by "
              "crystal with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2602_11709_amd import capi, synth
    capi.lib()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.config:
        legs = {"rocksalt": lambda: leg_rocksalt(20), "large_cells": lambda: leg_large_cells(3),
                "gradient_256": lambda: leg_gradients(5), "database_stream": leg_database}
        print(json.dumps({args.config: legs[args.config]()}), flush=True)
        return
    modes = {"auto": ("graph", "eager"), "graph": ("graph",), "eager": ("eager",)}[
        "eager" if args.no_graph else args.launch]
    batch = synth.triclinic_1024()
    rates = None if args.no_rates else rates_live()

    res = {}
    legs = [("mixed", "mixed", None)]
    if not args.no_fp64:
        # the plain path evaluates every reflection; with Friedel halving it
        # does the mixed path's work, so the two compare precision alone
        legs += [("fp64", "fp64", None), ("fp64_friedel", "fp64", True)]
    for name, precision, friedel in legs:
        p = Pipeline(batch, precision, friedel=friedel)
        with torch.cuda.stream(p.stream):
            # batch set-up, outside the timed region: the autotuner times the
            # structure-factor kernels' tile shapes and split-K thresholds on
            # the enumerated reflections
            p.enumerate()
            t0 = time.perf_counter()
            p.split = None if args.no_autotune else p.xb.autotune(p.refl)
            p.tune_ms = (time.perf_counter() - t0) * 1e3
            p.step()
        torch.cuda.synchronize()
        eager = p.outputs()
        if "graph" in modes:
            p.capture()
            for rep in range(3):  # every replay must reproduce the eager result bit for bit
                p.graph.replay()
                torch.cuda.synchronize()
                got = p.outputs()
                for k, v in eager.items():
                    if not torch.equal(v, got[k]):
                        raise RuntimeError(f"graph replay {rep} differs from eager in {k}")
        ms_by = {m: timed(p, args.steps, args.warmup, m == "graph") for m in modes}
        launch = min(ms_by, key=ms_by.get)
        ms = ms_by[launch]
        ro = p.refl.refl_offset.cpu().numpy()
        n_refl, terms = workload_stats(batch, ro)
        stages = {st: round(p.time_call(getattr(p, st), 10), 4)
                  for st in ("enumerate", "structure_factors", "merge", "pattern", "adjoint")}
        sf_ms = p.time_call(p.structure_factors, 20)
        eval_terms = terms // 2 if p.xb.friedel else terms
        res[name] = dict(p=p, ms=ms, n_refl=n_refl, terms=terms, eval_terms=eval_terms, stages=stages, sf_ms=sf_ms,
                         n_peaks=int(p.pk.peak_offset[-1]), eager=eager, launch=launch, ms_by=ms_by)
        if name != "mixed":
            del p.graph
            p.graph = None

    mx = res["mixed"]
    n_c = batch.n_crystals
    dbl_ms = None if args.no_doublet else doublet_ms(batch)
    front = None if args.no_doublet else frontend_rate(batch)
    fam = families_ms(mx["p"])
    value = n_c / (mx["ms"] * 1e-3)
    eval_terms = mx["eval_terms"]
    achieved = eval_terms / (mx["sf_ms"] * 1e-3)
    peak = term_peak_per_s()
    # the other long kernels of the step, timed per launch from the profiler's
    # kernel records over eager steps
    kus = kernel_device_us(torch, mx["p"].stream, mx["p"].step, 10,
                           ["k_sf<", "k_sf_bw<", "k_broaden_gather<", "k_broaden_adj<", "k_sort_merge<",
                            "k_peak_move", "k_peak_scan", "k_enum_fill", "k_enum_count", "k_enum_scan1",
                            "k_entry_prep<", "k_bw_finish"])
    pairs = entry_window_pairs(mx["p"])
    merge_bytes = 76 * mx["n_refl"]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["ms"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "triclinic_1024: 1024 synthetic triclinic crystals, a,b,c~U(3,15) A, angles U(60,120) "
                        "deg, 1-200 atoms log-uniform, 1-10 species each, B~U(0,2), Cu Ka 1.54184 A, "
                        "2theta 10-90 deg, merge tol 1e-5 deg, seed 1; step = enumerate + structure factors + "
                        "sort/merge/scale + 4001-point broadened pattern + its adjoint",
            "crystals": n_c, "atoms": int(batch.n_atoms), "reflections": mx["n_refl"], "peaks": mx["n_peaks"],
            "sf_terms": mx["terms"], "precision": "mixed: FP64 phase reduction, q, 2theta, LP, keys and "
            "intensities; FP32 sin/cos, scattering factors, weights and per-species sums, double across species",
            "launch": mx["launch"], "parallelism": "single GPU"},
        # every launch mode timed, each over its own --steps steps
        "ms_per_step_by_launch": {m: round(v, 6) for m, v in mx["ms_by"].items()},
        # structure-factor terms per second of the k_sf kernel: the evaluated
        # terms (one reflection of each Friedel pair) and, labelled effective,
        # all terms of the full sphere
        "sf_terms_per_s": round(achieved, 1),
        "sf_terms_per_s_effective": round(mx["terms"] / (mx["sf_ms"] * 1e-3), 1),
        "stages_ms": mx["stages"],
        "kernel_us": {k.rstrip("<"): round(v, 2) for k, v in kus.items()},
        "host_plan_ms": round(mx["p"].xb.plan_ms, 3),
        "batch_setup_ms": round(mx["p"].plan_ms, 3),
        "peak_families": fam,
        "frontend": front,
        "kalpha_doublet": None if dbl_ms is None else {
            "ms_per_step": round(dbl_ms, 6), "patterns_per_s": round(n_c / (dbl_ms * 1e-3), 1),
            "step": "Cu K-alpha1 + K-alpha2: enumerate, structure factors, merge, 4001-point pattern per line "
                    "(no adjoint)"},
        "autotune": None if mx["p"].split is None else {
            "split_atoms_forward": mx["p"].split[0], "split_atoms_adjoint": mx["p"].split[1],
            "reflections_per_lane": mx["p"].xb.sf_rpt, "ms": round(mx["p"].tune_ms, 1)},
        "roofline": {
            "kernel": "k_sf (mixed, Friedel-halved, keeping dF/ds^2)",
            "bound": "alu",
            "achieved": round(achieved / 1e9, 3),
            "peak": round(peak / 1e9, 3),
            "unit": "Gterm/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic_record(),
            "per_launch_terms": eval_terms,
            "avg_launch_ms": round(mx["sf_ms"], 5),
            "ops_per_term": UNIT_OPS["k_sf"],
            "peak_rates_per_cu_clk": {"f64": RATE_F64, "f32": RATE_F32, "trans": RATE_TRANS},
            "measured_term_mix": None if rates is None else round(rates["per_s"]["sf_term"] / 1e9, 3),
            "frac_of_measured_term_mix": None if rates is None else round(achieved / rates["per_s"]["sf_term"], 4),
        },
        "rooflines_other": {
            "k_sf_bw": None if "k_sf_bw<" not in kus else alu_roofline(
                "k_sf_bw", eval_terms, kus["k_sf_bw<"], "term",
                "profiler kernel records, 10 eager steps; every crystal of the workload takes the fused atom pass"),
            "k_broaden_gather": None if "k_broaden_gather<" not in kus else alu_roofline(
                "k_broaden_gather", pairs, kus["k_broaden_gather<"], "pair",
                "profiler kernel records, 10 eager steps; pairs = grid points within 8 sigma of each evaluated "
                "reflection"),
            "merge": {"kernels": "k_sort_merge (one launch for every crystal) + k_peak_move (numbering included "
                                 "up to 4096 crystals)",
                      "bound": "hbm", "achieved": round(merge_bytes / (mx["stages"]["merge"] * 1e-3) / 1e9, 1),
                      "peak": 8000.0, "unit": "GB/s",
                      "frac": round(merge_bytes / (mx["stages"]["merge"] * 1e-3) / 8e12, 4),
                      "per_launch_bytes": merge_bytes,
                      "bytes_per_reflection": "76: read 2theta and I (16), write perm (8), entries (6 per "
                                              "reflection), per peak (~half the reflections) staged record write "
                                              "and read and final write (~92)",
                      "timing": "merge stage, HIP events"},
        },
        "rates_measured": None if rates is None else {"per_cu_clk": rates["per_cu_clk"],
                                                       "copy_bytes_per_s": rates["copy_bytes_per_s"]},
    }
    if "fp64" in res:
        fp, ff = res["fp64"], res["fp64_friedel"]
        # error of the mixed path against the double path (which matches the oracle to ~1e-13)
        a, b = mx["eager"], fp["eager"]
        same = bool(torch.equal(a["mult"], b["mult"]))
        rel = None
        if same:
            offs = mx["p"].pk.peak_offset.cpu().numpy()
            rel = strong_peak_rel_err(offs, a["pk_i"].double().cpu().numpy(), b["pk_i"].cpu().numpy())
        for key, r in (("fp64", fp), ("fp64_friedel", ff)):
            line[key] = {"ms_per_step": round(r["ms"], 6), "patterns_per_s": round(n_c / (r["ms"] * 1e-3), 3),
                         "launch": r["launch"], "stages_ms": r["stages"], "sf_kernel_ms": round(r["sf_ms"], 5),
                         "sf_terms_per_s": round(r["eval_terms"] / (r["sf_ms"] * 1e-3), 1),
                         "evaluated_terms": r["eval_terms"]}
        # the same work (Friedel-halved) in both precisions: the precision's own effect
        line["speedup_mixed_vs_fp64"] = round(ff["ms"] / mx["ms"], 3)
        line["speedup_mixed_vs_fp64_sf_kernel"] = round(ff["sf_ms"] / mx["sf_ms"], 3)
        line["speedup_mixed_vs_fp64_all_reflections"] = round(fp["ms"] / mx["ms"], 3)
        line["mixed_vs_fp64_same_peaks"] = same
        line["mixed_vs_fp64_max_rel_err_strong_peaks"] = rel
    line["augmentation"] = augment_ms(mx["p"])  # last on this pipeline: it changes the buffers
    for key in list(res):
        if key != "mixed":
            del res[key]["p"]
    if not args.no_configs:
        line["recurrence"] = {"triclinic_1024": leg_recurrence(batch, 10),
                              "large_cells": leg_recurrence(synth.large_cells(), 3)}
    if not args.no_configs:
        line["configs"] = {"rocksalt": leg_rocksalt(20), "large_cells": leg_large_cells(3),
                           "gradient_256": leg_gradients(5), "database_stream": leg_database()}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
