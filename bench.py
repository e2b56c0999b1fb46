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
to fractional coordinates, B factors and lattice parameters).  The step is
captured once into a HIP graph and replayed; the timed region holds exactly
``--steps`` replays between two device synchronisations.

Printed: one JSON line (value = patterns per second of the mixed-precision
path), with the double-precision path timed the same way, the dominant
kernel's roofline and the oracle timed on the host as a CPU baseline.
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
# lane-operations per CU per clock on gfx950 (measured with microbenchmarks
# at 78% / 89% / 88-94% of these): FP32 VALU, FP64 VALU, transcendental
RATE_F32, RATE_F64, RATE_TRANS = 128.0, 64.0, 32.0
# per structure-factor term of the mixed kernel as the step runs it (keeping
# dF/ds^2 for the adjoint): phase h.x (3 FP64 FMA), reduction mod 1 and
# conversion (2 FP64-rate ops), sin + cos + exp (3 transcendental), weight
# exponent and two multiply-adds for F, one product and two multiply-adds for
# dF/ds^2 (6 FP32)
TERM_OPS = dict(f64=5, trans=3, f32=6)


def term_peak_per_s():
    clk_per_term = TERM_OPS["f64"] / RATE_F64 + TERM_OPS["trans"] / RATE_TRANS + TERM_OPS["f32"] / RATE_F32
    return N_CU * CLOCK_HZ / clk_per_term


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a graph replay")
    ap.add_argument("--no-fp64", action="store_true", help="skip the double-precision comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default structure-factor split thresholds")
    ap.add_argument("--no-doublet", action="store_true", help="skip the Cu K-alpha doublet forward timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters), then exit")
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

    def __init__(self, batch, precision, dy_seed=7):
        import torch
        from paper_2602_11709_amd.api import Grid, XrdBatch
        self.torch = torch
        self.grid = Grid(**GRID)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            t0 = time.perf_counter()
            # the step differentiates the pattern: the forward keeps dF/ds^2
            self.xb = XrdBatch(batch, precision=precision, keep_sf_derivs=True)
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
    import oracle
    cores = len(os.sched_getaffinity(0))
    threads = max(1, min(16, cores))
    # whole passes over the workload until about 20 s of CPU time (bounded)
    passes, wall = 0, 0.0
    t0 = time.perf_counter()
    while passes < 64 and (passes == 0 or wall * threads < 20.0):
        oracle.pattern_batch(batch, threads=threads, keep=False)
        passes += 1
        wall = time.perf_counter() - t0
    return {"value": passes * batch.n_crystals / wall, "unit": "patterns/s", "cores": threads, "kind": "oracle",
            "sample": f"{passes} passes over all {batch.n_crystals} crystals of the workload, forward pattern "
                      f"only (enumerate, structure factors, LP, sort, merge, scale; the oracle has no "
                      f"adjoint), plain FP64 C on {threads} OpenMP threads, {wall:.2f} s wall "
                      f"(~{wall * threads:.0f} thread-seconds)"}


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
    graph = not args.no_graph
    batch = synth.triclinic_1024()

    res = {}
    for precision in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        p = Pipeline(batch, precision)
        with torch.cuda.stream(p.stream):
            # batch set-up, outside the timed region: the split-K autotuner
            # times the structure-factor kernels on the enumerated reflections
            p.enumerate()
            t0 = time.perf_counter()
            p.split = None if args.no_autotune else p.xb.autotune(p.refl)
            p.tune_ms = (time.perf_counter() - t0) * 1e3
            p.step()
        torch.cuda.synchronize()
        eager = p.outputs()
        if graph:
            p.capture()
            for rep in range(3):  # every replay must reproduce the eager result bit for bit
                p.graph.replay()
                torch.cuda.synchronize()
                got = p.outputs()
                for k, v in eager.items():
                    if not torch.equal(v, got[k]):
                        raise RuntimeError(f"graph replay {rep} differs from eager in {k}")
        ms = timed(p, args.steps, args.warmup, graph)
        ro = p.refl.refl_offset.cpu().numpy()
        n_refl, terms = workload_stats(batch, ro)
        stages = {name: round(p.time_call(getattr(p, name), 10), 4)
                  for name in ("enumerate", "structure_factors", "merge", "pattern", "adjoint")}
        sf_ms = p.time_call(p.structure_factors, 20)
        res[precision] = dict(p=p, ms=ms, n_refl=n_refl, terms=terms, stages=stages, sf_ms=sf_ms,
                              n_peaks=int(p.pk.peak_offset[-1]), eager=eager)

    mx = res["mixed"]
    n_c = batch.n_crystals
    dbl_ms = None if args.no_doublet else doublet_ms(batch)
    fam = families_ms(mx["p"])
    aug = augment_ms(mx["p"])
    value = n_c / (mx["ms"] * 1e-3)
    eval_terms = mx["terms"] // 2 if mx["p"].xb.friedel else mx["terms"]
    achieved = eval_terms / (mx["sf_ms"] * 1e-3)
    peak = term_peak_per_s()
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
            "graph": graph, "parallelism": "single GPU"},
        "sf_terms_per_s": round(mx["terms"] / (mx["ms"] * 1e-3), 1),
        "stages_ms": mx["stages"],
        "host_plan_ms": round(mx["p"].xb.plan_ms, 3),
        "batch_setup_ms": round(mx["p"].plan_ms, 3),
        "peak_families": fam,
        "augmentation": aug,
        "kalpha_doublet": None if dbl_ms is None else {
            "ms_per_step": round(dbl_ms, 6), "patterns_per_s": round(n_c / (dbl_ms * 1e-3), 1),
            "step": "Cu K-alpha1 + K-alpha2: enumerate, structure factors, merge, 4001-point pattern per line "
                    "(no adjoint)"},
        "autotune": None if mx["p"].split is None else {
            "split_atoms_forward": mx["p"].split[0], "split_atoms_adjoint": mx["p"].split[1],
            "ms": round(mx["p"].tune_ms, 1)},
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
        },
    }
    if "fp64" in res:
        fp = res["fp64"]
        # error of the mixed path against the double path (which matches the oracle to ~1e-13)
        a, b = mx["eager"], fp["eager"]
        same = bool(torch.equal(a["mult"], b["mult"]))
        rel = None
        if same:
            pi, pr = a["pk_i"].double(), b["pk_i"]
            offs = mx["p"].pk.peak_offset.cpu().numpy()
            ref = pr.cpu().numpy()
            got = pi.cpu().numpy()
            worst = 0.0
            for c in range(n_c):
                s = slice(offs[c], offs[c + 1])
                if s.stop > s.start and ref[s].max() > 0:
                    strong = ref[s] >= 1e-3 * ref[s].max()
                    worst = max(worst, float(np.max(np.abs(got[s][strong] - ref[s][strong]) / ref[s][strong])))
            rel = worst
        line["fp64"] = {"ms_per_step": round(fp["ms"], 6), "patterns_per_s": round(n_c / (fp["ms"] * 1e-3), 3),
                        "stages_ms": fp["stages"], "sf_kernel_ms": round(fp["sf_ms"], 5),
                        "sf_terms_per_s_kernel": round(fp["terms"] / (fp["sf_ms"] * 1e-3), 1)}
        line["speedup_mixed_vs_fp64"] = round(fp["ms"] / mx["ms"], 3)
        line["mixed_vs_fp64_same_peaks"] = same
        line["mixed_vs_fp64_max_rel_err_strong_peaks"] = rel
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
