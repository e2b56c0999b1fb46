/*
 * xrd.h -- C ABI of the gfx950 kinematical powder-XRD library (libxrd.so).
 *
 * The library computes powder X-ray diffraction patterns of batches of
 * crystals on one MI355X GPU.  The method is the one the paper
 * (Rust-accelerated powder XRD, Section 2) accelerates on CPUs: generate the
 * reciprocal-lattice points inside the limiting sphere, evaluate each
 * reflection's structure factor as a sum over the atoms, apply the
 * Lorentz-polarisation and Debye-Waller corrections, and merge reflections
 * whose 2-theta agree within a tolerance into peaks.  The paper states the
 * problem as: lattice, atoms with species, occupancies and thermal factors,
 * wavelength, 2-theta range, and a scaled flag (Section 2, Fig. 1); the
 * output is a list of peaks with 2-theta, intensity, hkl list and
 * multiplicity, unfiltered (Section 2).
 *
 * Formulas (standard kinematical theory; the paper names the terms only):
 *   G* = inverse metric tensor, q = h^T G* h = 1/d^2, s^2 = q/4,
 *   2theta = 2 asin(lambda sqrt(q) / 2),
 *   f_t(s) = sum_{i=1..4} a_i exp(-b_i s^2) + c            (Cromer-Mann)
 *   F(hkl) = sum_j occ_j f_{t_j}(s) exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j))
 *   LP = (1 + cos^2 2theta) / (sin^2 theta cos theta),  I = |F|^2 LP.
 *
 * Conventions
 *  - Every call returns XRD_OK (0) or a negative XRD_ERR_* code and leaves a
 *    message for xrd_last_error() (thread-local).  No C++ exception crosses
 *    the ABI.
 *  - The caller owns every device buffer and the workspace; the batch
 *    handle owns only host memory.  The library never frees caller memory.
 *  - Device work is enqueued on the batch's stream in call order; no call
 *    synchronises the host except xrd_read_counts.  Buffers must stay valid
 *    until that stream work completes.
 *  - Outputs are CSR over crystals.  A crystal with no atoms or no reflection
 *    in its range is legal and yields an empty or all-zero segment.
 *  - Angles are in degrees, lengths in Angstrom, B in Angstrom^2.
 *  - Calls on one batch handle must not overlap from several host threads.
 */
#ifndef XRD_H
#define XRD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define XRD_OK 0
#define XRD_ERR_INVALID_ARG (-1)  /* null pointer, bad size, tolerance, range or wavelength */
#define XRD_ERR_INVALID_CELL (-2) /* lengths <= 0, angles outside (0,180), det(G)/(abc)^2 < 1e-3 */
#define XRD_ERR_CAPACITY (-3)     /* a size exceeds what the library's index types can hold */
#define XRD_ERR_HIP (-4)          /* a HIP runtime call failed (message names it) */
#define XRD_ERR_UNSUPPORTED (-5)  /* option combination not provided */

/* Arithmetic of the structure-factor, broadening and adjoint kernels. */
#define XRD_FP64 0  /* plain path: every step in double precision */
#define XRD_MIXED 1 /* phase h.x reduced mod 1 in double precision; sin/cos, scattering
                       factors and weights in single precision, summed in single
                       precision over at most 64 atoms of one species and those
                       partial sums added in double; q, 2theta, LP, merge keys and
                       intensities in double */

/* How xrd_structure_factors evaluates the sums over atoms (paper, Section 5
 * names reciprocal-space partitioning as the next step for large cells).
 * Both give the same structure factors up to rounding (within the bounds of
 * the precision). */
#define XRD_SF_DIRECT 0     /* every term e^{2 pi i (h x + k y + l z)} by sin/cos of its phase */
#define XRD_SF_RECURRENCE 1 /* along each row of constant (h, k) the reflections are cut into
                               segments of at most 8 consecutive l; per atom and segment the
                               weighted phasor occ e^{-B s^2} e^{2 pi i h.x} is evaluated exactly
                               at the first reflection and stepped to the next ones by a complex
                               product with r(l) e^{2 pi i z}, r(l) = e^{-B (q(l+1) - q(l))/4},
                               itself stepped by the constant ratio e^{-B G*33 / 2}; the segments
                               are rebuilt from the reflections by each call (workspace only) */
#define XRD_SF_AUTO 2       /* per crystal: the recurrence for crystals of at least 256 atoms whose
                               search box reaches |l| >= 12 (long rows), the direct sum for the
                               others (the two run concurrently); xrd_autotune picks the atom
                               threshold by timing */

typedef struct xrd_batch xrd_batch; /* opaque */

/* A batch of crystals.  Host arrays are read during xrd_batch_create only;
 * device arrays are read by the device calls and must stay valid until the
 * batch's work on the stream has completed. */
typedef struct {
    int64_t n_crystals;           /* >= 0 */
    int32_t n_species;            /* rows of sf_coeff, >= 1 */
    int32_t precision;            /* XRD_FP64 or XRD_MIXED */
    const double *lattice;        /* HOST [n_crystals*6]: a, b, c, alpha, beta, gamma */
    const int64_t *atom_offset;   /* HOST [n_crystals+1]: CSR offsets, atom_offset[0] == 0 */
    const double *two_theta_min;  /* HOST [n_crystals]: inclusive lower bound, >= 0 */
    const double *two_theta_max;  /* HOST [n_crystals]: inclusive upper bound, < 180 */
    double wavelength;            /* > 0 */
    double merge_tol;             /* > 0: anchor-rule merge tolerance in 2theta */
    double rel_threshold;         /* >= 0: drop merged peaks with I < rel_threshold * max I
                                     of their crystal (0 keeps every peak) */
    int32_t friedel;              /* 1: evaluate one reflection of each (h, -h) pair and copy
                                     the conjugate to its mate; 0: evaluate every reflection */
    int32_t grid_capacity;        /* largest n_points a broadened-pattern call on this batch
                                     will use; 0 selects 16384.  Sizes the workspace. */
    int32_t keep_sf_derivs;       /* 1: xrd_structure_factors also keeps dF/d(s^2) of the
                                     evaluated reflections in the workspace, and the next
                                     xrd_pattern_backward on the same enumeration, workspace and
                                     reflection arrays takes them from there instead of summing
                                     over the atoms again (forward and adjoint of the pattern
                                     share one pass over the atoms); 0: it does not.  Either way
                                     the results are the same up to rounding. */
    int32_t sf_method;            /* XRD_SF_DIRECT, XRD_SF_RECURRENCE or XRD_SF_AUTO */
    const double *frac;           /* DEVICE [N*3]: fractional x, y, z per atom */
    const int32_t *species;       /* DEVICE [N]: row of sf_coeff, 0 <= species < n_species */
    const double *occ;            /* DEVICE [N]: occupancy, >= 0 */
    const double *bfac;           /* DEVICE [N]: isotropic B */
    const double *sf_coeff;       /* DEVICE [n_species*9]: a1..a4, b1..b4, c */
    void *stream;                 /* hipStream_t; NULL = the null stream */
    int32_t forward_only;         /* 1: the batch never calls xrd_pattern_backward: its adjoint tables
                                     and buffers are neither built nor part of the workspace (a
                                     smaller plan and workspace for streams of forward patterns);
                                     xrd_pattern_backward then fails with XRD_ERR_UNSUPPORTED */
    int32_t sf_rpt;               /* tile shape of the direct structure-factor sums: reflections
                                     per lane, 1, 2 or 4 (a wavefront sums a tile of 64 times
                                     that); 0 selects 2 and lets xrd_autotune choose.  The
                                     workspace is sized for any shape. */
} xrd_batch_desc;

typedef struct {
    int64_t n_crystals;
    int64_t n_atoms;
    int64_t refl_capacity;   /* upper bound on the batch's reflections (sum of search boxes) */
    int64_t peak_capacity;   /* == refl_capacity */
    int64_t workspace_bytes; /* device workspace the batch needs, 256-byte aligned base */
    int64_t half_capacity;   /* upper bound on one-per-Friedel-pair reflections */
    int64_t noalloc_merge_bytes; /* scratch xrd_merge_peaks_noalloc needs for this batch (it
                                    runs only while this is <= XRD_NOALLOC_SCRATCH_BYTES) */
} xrd_sizes;

/* Reflection arrays (caller-owned device memory, capacity refl_capacity).
 * Crystal c owns [refl_offset[c], refl_offset[c+1]), listed in ascending
 * lexicographic (h, k, l) order; reflections i and (start + end - 1 - i) of a
 * crystal are Friedel mates. */
typedef struct {
    int16_t *h, *k, *l;
    double *q;           /* 1/d^2 */
    double *two_theta;   /* degrees */
    double *lp;          /* Lorentz-polarisation factor */
    int64_t *refl_offset;/* [n_crystals+1] */
} xrd_refl;

/* Merged peaks (caller-owned device memory, capacity peak_capacity).
 * Crystal c owns peaks [peak_offset[c], peak_offset[c+1]) in ascending 2theta.
 * perm lists every reflection in (2theta, h, k, l) order (global reflection
 * indices); a peak's members are perm[first .. first + mult). */
typedef struct {
    double *two_theta;   /* 2theta of the peak's first (smallest-angle) member */
    double *intensity;   /* sum of member intensities */
    double *scaled;      /* 100 * intensity / max intensity of the crystal (0 if that max is 0) */
    int32_t *mult;       /* number of member reflections */
    int64_t *first;      /* position in perm of the first member */
    int64_t *perm;       /* [refl_capacity] */
    int64_t *peak_offset;/* [n_crystals+1] */
} xrd_peaks;

/* Grid of a Gaussian-broadened pattern: x_g = t0 + g * dt, g in [0, n_points);
 * each reflection adds I exp(-(x - 2theta)^2 / (2 sigma^2)) / (sigma sqrt(2 pi))
 * at every grid point with |x - 2theta| <= window_sigmas * sigma. */
typedef struct {
    double t0, dt;
    int64_t n_points;
    double sigma, window_sigmas;
} xrd_grid;

/* Validate the batch and plan it on the host: metric inverses, search boxes,
 * capacities and launch tables.  Allocates host memory only and makes no HIP
 * call, so it also runs without a GPU.  On failure *out is NULL. */
int xrd_batch_create(const xrd_batch_desc *desc, xrd_batch **out);

/* Capacities and workspace size of a created batch (host only). */
int xrd_batch_sizes(const xrd_batch *b, xrd_sizes *out);

/* Change the cells of a planned batch (``lattice`` HOST [n_crystals*6], as in
 * the descriptor) without planning it again, for loops that refine the
 * lattice: each crystal keeps its search box, capacities and launch tables,
 * and takes the new inverse metric; the plan is copied into ``ws`` on the
 * batch's stream (enqueued, not waited for).  Fails with XRD_ERR_CAPACITY,
 * changing nothing, when a new cell needs a larger search box than the
 * batch was planned with (then create a new batch), and with
 * XRD_ERR_INVALID_CELL for an invalid cell.  The next device call must be
 * xrd_enumerate_hkl. */
int xrd_batch_set_lattice(xrd_batch *b, const double *lattice, void *ws);

/* Make ``stream`` (hipStream_t; NULL = the null stream) the batch's stream
 * for the calls that follow (host only).  Work already enqueued stays on the
 * previous stream; the caller orders the two (for instance, upload a batch's
 * tables on a copy stream, then set the compute stream). */
int xrd_batch_set_stream(xrd_batch *b, void *stream);

/* Copy the batch's launch tables into the workspace ``ws`` (device memory of
 * at least workspace_bytes, 256-byte aligned) on the batch's stream, and
 * wait for the copy.  Required once per workspace before the device calls
 * below, which then only launch kernels (so a caller may capture them into a
 * HIP graph and replay it). */
int xrd_batch_upload(xrd_batch *b, void *ws);

/* Reciprocal-lattice enumeration (paper, Section 2: lattice points inside
 * the physically accessible sphere): every integer (h, k, l) != 0 with
 * two_theta_min <= 2theta <= two_theta_max, with q, 2theta and LP, written
 * into ``r`` together with refl_offset.  Also packs the batch's atoms
 * (species-sorted copy) and, for XRD_MIXED, a single-precision copy of
 * sf_coeff into the workspace: xrd_structure_factors and
 * xrd_pattern_backward read those copies, so the device atom arrays (and
 * sf_coeff under XRD_MIXED) are read here and changes made to them later
 * take effect at the next call. */
int xrd_enumerate_hkl(xrd_batch *b, void *ws, const xrd_refl *r);

/* Structure factors (paper, Section 2: sum of atomic contributions for each
 * reflection, with Debye-Waller and Lorentz-polarisation factors) of every
 * reflection in ``r``.  A and B receive Re F and Im F (float under
 * XRD_MIXED, double under XRD_FP64; [refl_capacity]); I receives
 * |F|^2 LP in double ([refl_capacity]). */
int xrd_structure_factors(xrd_batch *b, void *ws, const xrd_refl *r, void *A, void *B, double *I);

/* Merge (paper, Section 2: merging of reflections within the angular
 * tolerance): sort each crystal's reflections by (2theta, h, k, l), then walk
 * them keeping a peak open while 2theta - 2theta(first member) < merge_tol;
 * scale to 0-100 and apply rel_threshold. */
int xrd_merge_peaks(xrd_batch *b, void *ws, const xrd_refl *r, const double *I, xrd_peaks *p);

/* Size of the fixed device scratch of xrd_merge_peaks_noalloc (64 MiB per GPU). */
#define XRD_NOALLOC_SCRATCH_BYTES 67108864

/* xrd_merge_peaks without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).
 * Same inputs, outputs and results as xrd_merge_peaks.  Its working storage
 * is a fixed scratch array of XRD_NOALLOC_SCRATCH_BYTES that the library
 * keeps on each GPU it runs on until the process ends; a batch whose merge
 * needs more than that (xrd_sizes.noalloc_merge_bytes, about 55 bytes per
 * reflection of capacity) is rejected with XRD_ERR_CAPACITY before any work is
 * enqueued.  Each call first copies the batch's merge tables into the scratch
 * (asynchronous copies from the handle's host memory on the batch's stream)
 * and runs every kernel on the batch's stream (no side streams).  All calls on
 * one GPU share that GPU's scratch, which keeps the last call's contents:
 * calls that overlap on one GPU (several host threads, or several streams
 * with work in flight) race and give wrong results; serialise them.  A later
 * xrd_pattern_forward / xrd_pattern_caglioti / xrd_pattern_backward on the
 * batch sorts again in its own workspace.  The first call on a device looks
 * up the scratch's device address (no allocation). */
int xrd_merge_peaks_noalloc(xrd_batch *b, const xrd_refl *r, const double *I, xrd_peaks *p);

/* Gaussian-broadened pattern y [n_crystals * n_points] (row per crystal) of
 * the reflections in ``r`` with intensities I; every reflection contributes
 * on its own (no merge).  Enumerate over the grid range widened by the
 * window on both sides so that no reflection reaching the grid is missed.
 * n_points must not exceed the batch's grid_capacity. */
int xrd_pattern_forward(xrd_batch *b, void *ws, const xrd_refl *r, const double *I,
                        const xrd_grid *g, double *y);

/* Adjoint of y(frac, lattice, bfac) = xrd_pattern_forward(enumerate, structure
 * factors): given dL/dy [n_crystals * n_points], writes dL/dfrac [N*3],
 * dL/dbfac [N] and dL/dlattice [n_crystals*6] (per degree for the angles).
 * The reflection set is held fixed (it is piecewise constant in the
 * lattice).  Uses the atoms packed by the last xrd_enumerate_hkl on ``ws``.
 * Device buffers, all double. */
int xrd_pattern_backward(xrd_batch *b, void *ws, const xrd_refl *r, const xrd_grid *g,
                         const double *dL_dy, double *dL_dfrac, double *dL_dbfac,
                         double *dL_dlattice);

/* Autotuner of the structure-factor launches (the batched execution of the
 * paper's structure-factor loops, Section 2 and Section 4.2): a crystal with
 * at least S atoms has each tile of its reflections summed by a block whose
 * four wavefronts split the atoms (split-K, partial sums added in a fixed
 * order), a smaller one by a single wavefront.  For the forward sum of
 * xrd_structure_factors and for the atom pass of xrd_pattern_backward
 * separately, times each candidate S (8 to 512, and no split) on this
 * batch's current reflections ``r`` (median of five launches) and keeps the
 * fastest in the batch and its launch tables in ``ws``.  Needs a prior
 * xrd_enumerate_hkl on ``ws`` and ``r``.  Synchronises the batch's stream
 * (a set-up call, not for graph capture); overwrites workspace scratch only,
 * so structure factors kept for the adjoint (keep_sf_derivs) must be
 * computed again.  The split changes only the summation order (results agree
 * to rounding).  ``split_out`` (optional, host [2]) receives the chosen
 * forward and adjoint S (INT32_MAX: no split).  Under XRD_SF_AUTO it first
 * times the per-crystal choice of the recurrence for atom thresholds of 64 to
 * 1024 (and never) and keeps the fastest; split_out must then hold 3 values,
 * the third the chosen atom threshold.  Unless the batch fixed its tile
 * shape (sf_rpt != 0), all of this is done for each shape (1, 2 and 4
 * reflections per lane) and the shape with the fastest forward plus adjoint
 * sum is kept with its splits; xrd_batch_get_sf_rpt reports it. */
int xrd_autotune(xrd_batch *b, void *ws, const xrd_refl *r, int32_t *split_out);

/* The batch's current tile shape of the direct structure-factor sums
 * (reflections per lane: 1, 2 or 4) into ``*rpt`` (host). */
int xrd_batch_get_sf_rpt(const xrd_batch *b, int32_t *rpt);

/* Experimental effects for ML training patterns (paper, Section 1: the
 * simulated patterns of ML training sets are modified with effects such as
 * preferred orientation and noise).
 *
 * Preferred orientation (March-Dollase; Dollase, J. Appl. Cryst. 19 (1986)
 * 267): multiplies each reflection's intensity I (in place, [refl_capacity])
 * by P = (r^2 cos^2(alpha) + sin^2(alpha) / r)^(-3/2), where
 * cos(alpha) = h^T G* hp / (|h| |hp|) and |v| = sqrt(v^T G* v).  hp (DEVICE
 * [n_crystals*3]) is each crystal's preferred direction as a reciprocal-
 * lattice vector in hkl components (need not be integer); march_r (DEVICE
 * [n_crystals]) its March parameter (1: random powder, < 1 plates, > 1
 * needles).  A crystal with march_r <= 0 or a zero hp is left unchanged.
 * Apply it between xrd_structure_factors and xrd_merge_peaks or
 * xrd_pattern_forward. */
int xrd_preferred_orientation(xrd_batch *b, void *ws, const xrd_refl *r, const double *hp,
                              const double *march_r, double *I);

/* Equivalence rules of xrd_peak_families. */
#define XRD_FAMILY_INDICES 0 /* equal multisets of |h|, |k|, |l|; of |h|, |k|, |h+k|, |l| on a
                                hexagonal lattice (a = b, alpha = beta = 90, gamma = 120) */
#define XRD_FAMILY_LATTICE 1 /* related by a point operation M of the lattice: hkl -> M hkl with
                                M integer, entries in {-1, 0, 1}, det M = +-1, M^T G* M = G* */

/* Families of symmetry-equivalent reflections in each merged peak (paper,
 * Section 2: grouping of symmetry-equivalent reflections; Section 3: a
 * peak's hkl list gives families with a multiplicity each).  The batch
 * carries no space group, so ``rule`` picks the equivalence (XRD_FAMILY_*);
 * metric equalities hold within 1e-6 of the largest diagonal entry of G*.
 * Reads r's h, k, l and p's first, mult, perm and peak_offset from a
 * completed xrd_merge_peaks.  Walking a peak's members in their order
 * (positions first .. first + mult - 1 of perm), a member joins the family of
 * an earlier equivalent member or opens the next family.  Outputs (DEVICE,
 * caller-owned):
 *   n_families [peak_capacity]: families of each peak;
 *   family_of [refl_capacity]: at each member position, its family's number
 *     within its peak (0-based);
 *   family_label, family_mult [refl_capacity]: family f of the peak whose
 *     first member sits at position first sits at position first + f: the
 *     global reflection index of its lexicographically largest (h, k, l)
 *     member, and its number of members.
 * Positions of perm outside the kept peaks are left unchanged.  One thread
 * per peak: cost grows with the square of the members per peak. */
int xrd_peak_families(xrd_batch *b, void *ws, const xrd_refl *r, const xrd_peaks *p, int32_t rule,
                      int32_t *n_families, int32_t *family_of, int64_t *family_label, int32_t *family_mult);

/* One emission line's peaks for xrd_combine_lines: ``peaks`` from a
 * completed xrd_merge_peaks (two_theta, intensity, mult, first, perm and
 * peak_offset are read; DEVICE) on a batch of that line's wavelength, ``q``
 * (DEVICE) the reflections' q of the same batch, ``weight`` the line's
 * relative intensity. */
typedef struct {
    const xrd_peaks *peaks;
    const double *q;
    double weight;
} xrd_line;

/* Combined peak list of one or two emission lines (all DEVICE, caller-owned,
 * capacity >= the two lines' peaks together). */
typedef struct {
    double *two_theta;     /* degrees, ascending within each crystal */
    double *intensity;     /* weight x the line's peak intensity */
    double *scaled;        /* 100 x intensity / the crystal's largest over both lines (0 if that is 0) */
    int32_t *mult;         /* member reflections of the peak */
    double *d;             /* interplanar spacing 1 / sqrt(q) of the peak's first member, Angstrom */
    int32_t *line;         /* 0: line0, 1: line1 */
    int64_t *source;       /* the peak's index in its line's peak arrays */
    int64_t *peak_offset;  /* [n_crystals + 1]: the two lines' offsets added */
} xrd_line_peaks;

/* The calculator's peak list for a doublet (paper, Section 2: the peaks'
 * 2theta, intensity, interplanar spacing and multiplicity, scaled to 0-100 on
 * request; the K-alpha1 and K-alpha2 lines are computed as two batches): per
 * crystal, the peaks of line0 and of line1 (NULL: line0 alone) in one list in
 * ascending 2theta (at equal 2theta line0's first, each line's own order
 * kept), intensities weighted, scaled jointly by the crystal's largest
 * weighted intensity, with d and the source of each peak.  Enqueued on
 * ``stream`` (hipStream_t; NULL = the null stream).  No workspace. */
int xrd_combine_lines(int64_t n_crystals, const xrd_line *line0, const xrd_line *line1, xrd_line_peaks *out,
                      void *stream);

/* Broadened pattern y [n_crystals * n_points] with widths that grow with
 * angle (Caglioti, Paoletti and Ricci, Nucl. Instrum. 3 (1958) 223) and
 * pseudo-Voigt profiles (paper, Section 1: peak broadening among the
 * experimental effects of ML training patterns): each reflection adds its
 * intensity times eta L + (1 - eta) G, a unit-area Lorentzian L and a
 * unit-area Gaussian G of one FWHM, FWHM^2 = U tan^2(theta) + V tan(theta)
 * + W (degrees^2, theta = 2theta / 2), sigma = FWHM / (2 sqrt(2 ln 2)), at
 * the grid points with |x - 2theta| <= window_sigmas sigma (both components
 * cut there); a reflection with FWHM^2 <= 0 adds nothing.  0 <= eta <= 1
 * (0: Gaussian).  The grid's t0, dt, n_points and window_sigmas apply; its sigma is
 * not used (any positive value).  Sums in double precision, each point over
 * its reflections in 2theta order (deterministic); forward only.  Under
 * XRD_MIXED each profile value is a single-precision exp2 and reciprocal
 * (relative error below 1e-5 per term), as in xrd_pattern_forward; under
 * XRD_FP64 all double. */
int xrd_pattern_caglioti(xrd_batch *b, void *ws, const xrd_refl *r, const double *I, const xrd_grid *g,
                         double U, double V, double W, double eta, double *y);

/* Noise on broadened patterns y (DEVICE [n_crystals*n_points], in place):
 * y += (rel sqrt(max(y, 0)) + abs) z, a counting-statistics term and a flat
 * term, with z the standard normal variate number n = c n_points + g of the
 * stream ``seed``: outputs 2n+1 and 2n+2 of SplitMix64 (Steele, Lea and
 * Flood, OOPSLA 2014) seeded with ``seed`` give u1, u2 = (top 53 bits + 1/2)
 * 2^-53, and z = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller).  The same seed
 * gives the same noise.  1 <= n_points <= grid_capacity; rel, abs >= 0. */
int xrd_pattern_noise(xrd_batch *b, int64_t n_points, uint64_t seed, double rel, double abs, double *y);

/* Wait for the batch's stream and copy refl_offset and peak_offset
 * ([n_crystals+1] each; either may be NULL) to host memory. */
int xrd_read_counts(xrd_batch *b, const xrd_refl *r, const xrd_peaks *p,
                    int64_t *host_refl_offset, int64_t *host_peak_offset);

/* Free the handle, and the two streams and three events it keeps for work
 * that runs beside the caller's stream inside a call (created at the first
 * sort on a device; the batch's work must have completed).  NULL is ignored. */
void xrd_batch_destroy(xrd_batch *b);

/* Message of the last failed call on this thread ("" if none). */
const char *xrd_last_error(void);

/* Library version string. */
const char *xrd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XRD_H */
