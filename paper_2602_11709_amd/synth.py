"""Seeded synthetic crystal batches.

This module only draws inputs: lattices, atom lists, species tables, wavelength
and 2-theta ranges.  It contains none of the diffraction arithmetic, so both the
GPU path and the CPU oracle may import it without sharing any computation.

The recipes stand in for the structure databases the paper benchmarks on
(MC3D and COD, Section 4), which are not available here.  Every draw comes from
``numpy.random.default_rng(seed)`` (PCG64) in the order written below, so a
batch is reproducible from its seed alone.

Species are synthetic four-Gaussian-plus-constant scattering-factor curves
(the Cromer-Mann form): nine coefficients a1..a4, b1..b4, c with
a_i ~ U(0.5, 6), b_i ~ U(0.5, 60) A^2, c ~ U(0, 1), drawn per species in the
order a (4 values), b (4 values), c.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

CU_KA = 1.54184  # A, single line (no K-alpha doublet)
MO_KA = 0.71073  # A, single line

# A cell is rejected when 1 - sum cos^2 + 2 prod cos (= det(G)/(abc)^2) is
# below this value: such cells are nearly flat.
CELL_DET_MIN = 1e-3


@dataclasses.dataclass
class CrystalBatch:
    """A batch of crystals in CSR layout.

    lattice      (n_c, 6) float64: a, b, c in Angstrom; alpha, beta, gamma in degrees
    atom_offset  (n_c + 1,) int64: atoms of crystal c are [atom_offset[c], atom_offset[c+1])
    frac         (N, 3) float64: fractional coordinates
    species      (N,) int32: row of ``sf_coeff``
    occ          (N,) float64: site occupancy
    bfac         (N,) float64: isotropic Debye-Waller B, Angstrom^2
    sf_coeff     (S, 9) float64: a1..a4, b1..b4, c per species
    wavelength   float, Angstrom
    two_theta_min, two_theta_max  (n_c,) float64, degrees
    merge_tol    float, degrees
    """

    name: str
    lattice: np.ndarray
    atom_offset: np.ndarray
    frac: np.ndarray
    species: np.ndarray
    occ: np.ndarray
    bfac: np.ndarray
    sf_coeff: np.ndarray
    wavelength: float
    two_theta_min: np.ndarray
    two_theta_max: np.ndarray
    merge_tol: float = 1e-5

    @property
    def n_crystals(self) -> int:
        return int(self.lattice.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.frac.shape[0])

    @property
    def n_species(self) -> int:
        return int(self.sf_coeff.shape[0])

    def atoms_of(self, c: int) -> slice:
        return slice(int(self.atom_offset[c]), int(self.atom_offset[c + 1]))

    def counts(self) -> np.ndarray:
        return np.diff(self.atom_offset)

    def subset(self, idx) -> "CrystalBatch":
        """Crystals ``idx`` (in that order) as a new batch sharing the species table."""
        idx = [int(i) for i in idx]
        parts = [self.atoms_of(c) for c in idx]
        sizes = np.array([p.stop - p.start for p in parts], dtype=np.int64)
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        cat = (lambda a: np.concatenate([a[p] for p in parts]) if parts else a[:0])
        return CrystalBatch(
            name=f"{self.name}[subset]",
            lattice=self.lattice[idx].copy(),
            atom_offset=off,
            frac=cat(self.frac).reshape(-1, 3),
            species=cat(self.species).astype(np.int32),
            occ=cat(self.occ),
            bfac=cat(self.bfac),
            sf_coeff=self.sf_coeff.copy(),
            wavelength=self.wavelength,
            two_theta_min=self.two_theta_min[idx].copy(),
            two_theta_max=self.two_theta_max[idx].copy(),
            merge_tol=self.merge_tol,
        )


def species_pool(rng: np.random.Generator, n: int) -> np.ndarray:
    """``n`` synthetic species, coefficients drawn a(4), b(4), c per species."""
    out = np.empty((n, 9), dtype=np.float64)
    for s in range(n):
        out[s, 0:4] = rng.uniform(0.5, 6.0, 4)
        out[s, 4:8] = rng.uniform(0.5, 60.0, 4)
        out[s, 8] = rng.uniform(0.0, 1.0)
    return out


def cell_flatness(alpha, beta, gamma) -> float:
    """det(G)/(abc)^2 of a cell with these angles (degrees): the rejection test."""
    ca, cb, cg = (math.cos(math.radians(v)) for v in (alpha, beta, gamma))
    return 1.0 - ca * ca - cb * cb - cg * cg + 2.0 * ca * cb * cg


def _angles(rng, lo=60.0, hi=120.0):
    while True:
        ang = rng.uniform(lo, hi, 3)
        if cell_flatness(*ang) >= CELL_DET_MIN:
            return ang


def _assemble(name, lattices, atoms, sf_coeff, wavelength, tmin, tmax, tol=1e-5):
    n_c = len(lattices)
    counts = np.array([len(a[0]) for a in atoms], dtype=np.int64)
    off = np.zeros(n_c + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    if n_c:
        frac = np.concatenate([a[0] for a in atoms]).reshape(-1, 3)
        spec = np.concatenate([a[1] for a in atoms]).astype(np.int32)
        occ = np.concatenate([a[2] for a in atoms]).astype(np.float64)
        bfac = np.concatenate([a[3] for a in atoms]).astype(np.float64)
    else:
        frac = np.zeros((0, 3))
        spec = np.zeros(0, np.int32)
        occ = np.zeros(0)
        bfac = np.zeros(0)
    return CrystalBatch(
        name=name,
        lattice=np.asarray(lattices, dtype=np.float64).reshape(n_c, 6),
        atom_offset=off,
        frac=np.ascontiguousarray(frac, dtype=np.float64),
        species=spec,
        occ=occ,
        bfac=bfac,
        sf_coeff=np.ascontiguousarray(sf_coeff, dtype=np.float64),
        wavelength=float(wavelength),
        two_theta_min=np.full(n_c, float(tmin)),
        two_theta_max=np.full(n_c, float(tmax)),
        merge_tol=float(tol),
    )


def rocksalt(seed: int = 0, a: float = 5.64, bfac: float = 0.5) -> CrystalBatch:
    """One rock-salt-type cubic cell: species A on the four fcc sites, species B
    on the same sites shifted by (1/2, 0, 0); two synthetic species drawn from
    ``seed`` (A first, then B); B = 0.5 A^2, occupancy 1, Cu K-alpha, 2-theta 0-90."""
    rng = np.random.default_rng(seed)
    coeff = species_pool(rng, 2)
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]], dtype=np.float64)
    sites_b = np.mod(fcc + np.array([0.5, 0.0, 0.0]), 1.0)
    frac = np.concatenate([fcc, sites_b])
    spec = np.array([0] * 4 + [1] * 4, dtype=np.int32)
    atoms = [(frac, spec, np.ones(8), np.full(8, bfac))]
    return _assemble("rocksalt", [[a, a, a, 90.0, 90.0, 90.0]], atoms, coeff, CU_KA, 0.0, 90.0)


def random_triclinic(seed: int, n_crystals: int, *, len_lo=3.0, len_hi=15.0,
                     atoms_lo=1, atoms_hi=200, species_per_crystal=10, pool=64,
                     wavelength=CU_KA, tmin=10.0, tmax=90.0,
                     name="triclinic") -> CrystalBatch:
    """Uneven batch of triclinic crystals.

    Draw order: species pool (``pool`` species); then per crystal: a, b, c ~
    U(len_lo, len_hi); angles ~ U(60, 120) deg redrawn until the cell passes the
    flatness test; atom count round(exp(U(ln atoms_lo, ln atoms_hi))) (log-
    uniform); k ~ U{1 .. min(species_per_crystal, N)} species chosen from the
    pool without replacement; per atom: species uniform over the k, fractional
    coordinates U[0,1)^3, B ~ U(0, 2) A^2; occupancy 1.
    """
    rng = np.random.default_rng(seed)
    coeff = species_pool(rng, pool)
    lattices, atoms = [], []
    for _ in range(n_crystals):
        lengths = rng.uniform(len_lo, len_hi, 3)
        ang = _angles(rng)
        n = int(round(math.exp(rng.uniform(math.log(atoms_lo), math.log(atoms_hi)))))
        n = max(atoms_lo, min(atoms_hi, n))
        k = int(rng.integers(1, min(species_per_crystal, n) + 1))
        chosen = rng.choice(pool, size=k, replace=False)
        spec = chosen[rng.integers(0, k, n)]
        frac = rng.uniform(0.0, 1.0, (n, 3))
        bf = rng.uniform(0.0, 2.0, n)
        lattices.append([*lengths, *ang])
        atoms.append((frac, spec, np.ones(n), bf))
    return _assemble(name, lattices, atoms, coeff, wavelength, tmin, tmax)


def triclinic_1024(seed: int = 1) -> CrystalBatch:
    """1024 triclinic crystals, 1-200 atoms (log-uniform), 1-10 species each,
    a, b, c ~ U(3, 15) A, Cu K-alpha, 2-theta 10-90."""
    return random_triclinic(seed, 1024, name="triclinic_1024")


def large_cells(seed: int = 2, n_crystals: int = 16) -> CrystalBatch:
    """Large-cell stress batch: half monoclinic (alpha = gamma = 90, beta ~
    U(90, 120)), half triclinic; a, b, c ~ U(30, 50) A; 2000-5000 atoms; a pool
    of 20 species, each atom uniform over the pool; occupancy ~ U(0.5, 1);
    B ~ U(0, 2); Cu K-alpha; 2-theta 5-120.

    Draw order: pool; then per crystal: lengths, angles (beta only when
    monoclinic), N ~ U{2000..5000}, per-atom species, fractional coordinates,
    occupancy, B."""
    rng = np.random.default_rng(seed)
    coeff = species_pool(rng, 20)
    lattices, atoms = [], []
    for c in range(n_crystals):
        lengths = rng.uniform(30.0, 50.0, 3)
        if c < n_crystals // 2:
            ang = np.array([90.0, rng.uniform(90.0, 120.0), 90.0])
        else:
            ang = _angles(rng)
        n = int(rng.integers(2000, 5001))
        spec = rng.integers(0, 20, n)
        frac = rng.uniform(0.0, 1.0, (n, 3))
        occ = rng.uniform(0.5, 1.0, n)
        bf = rng.uniform(0.0, 2.0, n)
        lattices.append([*lengths, *ang])
        atoms.append((frac, spec, occ, bf))
    return _assemble("large_cells", lattices, atoms, coeff, CU_KA, 5.0, 120.0)


def database_stream(seed: int = 3, n_crystals: int = 100_000, pool: int = 96,
                    wavelength=MO_KA, tmin=2.0, tmax=60.0) -> CrystalBatch:
    """Database-scale stream: N = clip(round(LogNormal(ln 20, 1.0)), 1, 1000)
    atoms; each length = 2.6 A * N^(1/3) * U(0.8, 1.2); angles ~ U(60, 120) with
    the flatness test; k ~ U{1..min(10, N)} species; B ~ U(0, 2); occupancy 1.
    The paper's benchmark settings (Mo K-alpha, 2-theta 2-60) are the default.

    Draw order per crystal: N, lengths (3), angles, k, species choice, per-atom
    species, fractional coordinates, B."""
    rng = np.random.default_rng(seed)
    coeff = species_pool(rng, pool)
    lattices, atoms = [], []
    for _ in range(n_crystals):
        n = int(np.clip(round(rng.lognormal(math.log(20.0), 1.0)), 1, 1000))
        lengths = 2.6 * n ** (1.0 / 3.0) * rng.uniform(0.8, 1.2, 3)
        ang = _angles(rng)
        k = int(rng.integers(1, min(10, n) + 1))
        chosen = rng.choice(pool, size=k, replace=False)
        spec = chosen[rng.integers(0, k, n)]
        frac = rng.uniform(0.0, 1.0, (n, 3))
        bf = rng.uniform(0.0, 2.0, n)
        lattices.append([*lengths, *ang])
        atoms.append((frac, spec, np.ones(n), bf))
    return _assemble("database_stream", lattices, atoms, coeff, wavelength, tmin, tmax)


@dataclasses.dataclass
class GradientProblem:
    """Inputs of the differentiable broadened-pattern workload.

    ``batch`` is the structure to optimise, ``target`` the perturbed structure
    whose broadened pattern is the regression target.  The grid is
    ``grid_t0 + g * grid_dt`` for g in [0, grid_n) (degrees) and the Gaussian
    width is ``sigma`` degrees with a window of ``window_sigmas`` widths.
    Reflections are enumerated over the grid range widened by the window on
    both sides, so no reflection that can reach the grid is missed."""

    batch: CrystalBatch
    target: CrystalBatch
    grid_t0: float
    grid_dt: float
    grid_n: int
    sigma: float
    window_sigmas: float


def gradient_problem(seed: int = 4, n_crystals: int = 256, atoms_lo=50, atoms_hi=500,
                     grid_n=4001, t0=10.0, t1=90.0, sigma=0.1, window_sigmas=8.0,
                     pool=64) -> GradientProblem:
    """256 crystals of 50-500 atoms, lattices by the database-stream rule,
    Cu K-alpha, a 4001-point grid over 10-90 deg, sigma = 0.1 deg.

    Draw order: pool; per crystal: N ~ U{atoms_lo..atoms_hi}, lengths, angles,
    k, species, per-atom species, fractional coordinates, B; then, for the
    target, per crystal: fractional shifts N(0, 0.005) (wrapped into [0,1)),
    length factors 1 + N(0, 0.005), angle shifts N(0, 0.2) deg, B shifts
    N(0, 0.05) clipped at 0."""
    rng = np.random.default_rng(seed)
    coeff = species_pool(rng, pool)
    pad = window_sigmas * sigma
    lattices, atoms = [], []
    for _ in range(n_crystals):
        n = int(rng.integers(atoms_lo, atoms_hi + 1))
        lengths = 2.6 * n ** (1.0 / 3.0) * rng.uniform(0.8, 1.2, 3)
        ang = _angles(rng)
        k = int(rng.integers(1, min(10, n) + 1))
        chosen = rng.choice(pool, size=k, replace=False)
        spec = chosen[rng.integers(0, k, n)]
        frac = rng.uniform(0.0, 1.0, (n, 3))
        bf = rng.uniform(0.0, 2.0, n)
        lattices.append([*lengths, *ang])
        atoms.append((frac, spec, np.ones(n), bf))
    batch = _assemble("gradient", lattices, atoms, coeff, CU_KA, t0 - pad, t1 + pad)

    tlat, tatoms = [], []
    for c in range(n_crystals):
        sl = batch.atoms_of(c)
        n = sl.stop - sl.start
        frac = np.mod(batch.frac[sl] + rng.normal(0.0, 0.005, (n, 3)), 1.0)
        lat = batch.lattice[c].copy()
        lat[:3] *= 1.0 + rng.normal(0.0, 0.005, 3)
        lat[3:] += rng.normal(0.0, 0.2, 3)
        bf = np.maximum(batch.bfac[sl] + rng.normal(0.0, 0.05, n), 0.0)
        tlat.append(lat)
        tatoms.append((frac, batch.species[sl], batch.occ[sl], bf))
    target = _assemble("gradient_target", tlat, tatoms, coeff, CU_KA, t0 - pad, t1 + pad)
    dt = (t1 - t0) / (grid_n - 1)
    return GradientProblem(batch, target, t0, dt, grid_n, sigma, window_sigmas)
