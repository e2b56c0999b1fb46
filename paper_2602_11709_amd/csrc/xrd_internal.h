// Internal layout shared by the host planner and the gfx950 kernels of libxrd.
//
// The host plans a batch once (metric inverses, search boxes, capacities and
// launch tables); the plan is copied into the caller's workspace and every
// kernel reads it from there.  All device scratch lives in that workspace at
// offsets fixed by the plan, so no call allocates device memory and every
// launch has a grid size known on the host (HIP-graph friendly).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xrd {

// Work granularity.
constexpr int kEnumRows = 32;     // most (h, k) rows of a half search box per enumeration chunk, one per lane
constexpr int kEnumCand = 256;    // candidate points a chunk takes before the next chunk starts (one fill round)
constexpr int kSortChunk = 1024;  // reflections per sort/merge block (256 threads x 4)
constexpr int kBinDiv = 4;        // merge-sort bins per crystal = capacity / kBinDiv
constexpr int kHalfChunk = 2048;  // reflections per adjoint chunk
constexpr int kEntBlock = 1024;   // entries per block of the broadening's entry preparation and adjoint
constexpr int kScanBlock = 2048;  // elements per scan block (256 threads x 8)
constexpr int kAtomBlock = 256;   // atoms per adjoint block
constexpr int kSfThreads = 256;   // threads per block of the structure-factor kernels
// Tile shape of the direct structure-factor kernels: reflections per lane
// (1, 2 or 4; a tile is 64 times that), per batch; the default, and the
// finest one, for which the workspace's per-tile tables are sized.
constexpr int kSfRptDefault = 2;
constexpr int kSfRptMin = 1;
constexpr int kFusedMaxAtoms = 512;  // crystals up to this size take the fused atom-gradient path
// Split-K of the structure-factor kernels: crystals with at least this many
// atoms get a block per tile, whose four wavefronts split the atom sum; the
// others a wavefront per tile.  Defaults for the forward sum and for the
// adjoint's atom pass; xrd_autotune picks them per batch by timing.
constexpr int kSplitFwd = 64;
constexpr int kSplitBw = 48;
constexpr int kTinySort = 1024;      // Friedel-positive reflections sorted in LDS by one 256-thread block
constexpr int kSmallSort = 4096;     // ... by one 1024-thread block
constexpr int kMidSort = 6144;       // ... by one 1024-thread block; larger crystals sort in global memory
// Crystals whose reflection capacity exceeds kBigSort sort in global memory
// over many blocks (kBigChunk reflections, sorted positions or peak slots
// each) when they have more than 2 kMidSort reflections; the others in
// global memory take one block (they must fill more than half their search
// box, which a sphere shell in a box rarely does).  2 kBigSort bounds the
// capacity of 15 A cells under Cu K-alpha to 90 deg, so such batches launch
// no many-block kernels.
constexpr int64_t kBigSort = 24576;
constexpr int kBigChunk = 4096;
constexpr int kSpanPts = 16;         // grid points per span of the broadening gather (a quarter wavefront)
constexpr int kRecLen = 8;           // reflections per segment of the row-recurrence structure factors
constexpr int kRecMinAtoms = 256;    // XRD_SF_AUTO: default atom threshold of the recurrence
constexpr int kRecMinRow = 12;       // XRD_SF_AUTO: the recurrence needs |l| up to at least this in the search box
// Device scratch of the allocation-free merge entry point (one array per GPU).
constexpr int64_t kNoallocBytes = (int64_t)64 << 20;

// Per-crystal plan (device copy in the workspace), 256 bytes.
struct alignas(16) CrystalPlan {
  double gs[6];       // G* as [11, 22, 33, 12, 13, 23]
  double lat[6];      // a, b, c (A), alpha, beta, gamma (deg)
  double tmin, tmax;  // inclusive 2theta range (deg)
  double qlo, qhi;    // conservative q prefilter: points outside never pass the 2theta test
  double bin_scale;   // merge-sort bins per degree
  int32_t H, K, L;    // search box half extents
  int32_t n_bins;
  int64_t half_box;   // points of the search box above the origin: ((2H+1)(2K+1)(2L+1)-1)/2
  int64_t enum_chunk_begin;
  int32_t enum_chunks;  // runs of consecutive rows of the half box (EnumChunk)
  int32_t n_hchunks;  // adjoint chunks at capacity
  int64_t atom_begin, atom_end;
  int64_t run_begin;  // first slot of this crystal's species-run table (capacity min(S, N))
  int64_t bin_begin;
  int64_t sort_chunk_begin;
  int64_t hchunk_begin;  // first adjoint chunk (global id)
  int64_t part_begin;    // first adjoint partial row: rows = n_hchunks * N
  int32_t sort_chunks;
  int16_t fused;       // 1: atom gradients reduced inside the reflection-major adjoint
  int16_t sf_tile;     // reflections per structure-factor tile (64 x reflections per lane)
  int64_t pf_begin;    // first row of the fused adjoint partials: rows = n_tiles * N
  int32_t n_tiles;     // structure-factor tiles at capacity
  int32_t tile_begin;  // first row of this crystal's per-tile dL/dG* rows
};
static_assert(sizeof(CrystalPlan) == 256, "CrystalPlan layout");

// Packed atom, species-sorted within each crystal (48 bytes).
struct alignas(16) AtomRec {
  double x, y, z;
  double occ, bfac;
  float log2occ;   // log2(occ) (mixed path weight exponent)
  float bl2e;      // B * log2(e)
};
static_assert(sizeof(AtomRec) == 48, "AtomRec layout");

// Per-atom factors of the row recurrence (48 bytes, parallel to AtomRec):
// the phase step e^{2 pi i z} = (zc, zs) along l and rho = e^{-B G*33 / 2},
// the ratio of successive Debye-Waller steps along l, in double and single
// precision.
struct alignas(16) AtomRot {
  double zc, zs, rho;
  float zcf, zsf, rhof, pad;
};
static_assert(sizeof(AtomRot) == 48, "AtomRot layout");

// Cromer-Mann coefficients of one species in single precision, in the form
// the mixed-precision kernels evaluate them (64 bytes, one scalar load):
//   f(s^2) = c + sum_i a_i 2^(nbl_i s^2),  df/ds^2 = sum_i nab_i 2^(nbl_i s^2),
// with nbl_i = -b_i log2(e) and nab_i = -a_i b_i rounded once from double.
// Point operations of one crystal's lattice for the grouping of equivalent
// reflections: op[o] packs the 3x3 matrix M (entries in {-1, 0, 1}, row r,
// column j at bits 6r + 2j as M_rj + 1); hex is 1 on a hexagonal lattice.
struct alignas(16) FamOps {
  int32_t n_ops, hex, pad[2];
  uint32_t op[48];
};

struct alignas(16) CoeffF {
  float a[4], nbl[4], nab[4];
  float c, pad[3];
};
static_assert(sizeof(CoeffF) == 64, "CoeffF layout");

// A run of same-species atoms: [begin, end) in the packed array.
struct alignas(16) SpeciesRun {
  int32_t begin, end, species, local;  // local = run index within the crystal
};

// Enumeration work unit: rows [row_begin, row_begin + n_rows) of a crystal's
// half box (n_rows <= kEnumRows), cut so that the chunks' candidate counts
// stay near kEnumCand.
struct EnumChunk {
  int32_t crystal, row_begin, n_rows, pad;
};

// Broadening work unit: chunk of kHalfChunk entries of one crystal.
struct HChunk {
  int32_t crystal;
  int32_t chunk;
};

// Unit of the many-block global-memory sort: chunk ``chunk`` of crystal
// ``crystal``, whose n chunks hold the slots first .. first + n - 1 of the
// per-chunk count and offset arrays, whose nb 2theta buckets have their
// per-chunk counts at hbase + chunk nb + bucket and their offsets at bbase +
// bucket (the crystal list uses chunk = 0).
struct BigChunk {
  int32_t crystal, chunk, first, n, nb, pad;
  int64_t hbase, bbase;
};
static_assert(sizeof(BigChunk) == 40, "BigChunk layout");
constexpr int kBigBucketsMax = 8192;  // 2theta buckets of a crystal in the many-block sort, at most

// Structure-factor work item: a tile of reflections of one crystal, with
// the crystal's atom range and species-run slots (from the plan), so that a
// wavefront's atom loads do not wait for the plan (32 bytes, one scalar load).
struct alignas(32) SfItem {
  int32_t crystal;
  int32_t tile;
  int32_t atom_begin, atom_end;  // packed atoms [atom_begin, atom_end)
  int32_t run_begin;             // first slot of the crystal's species-run table
  int32_t tail;                  // 1: take tiles tile, tile + 1, ... up to the crystal's last one
  int32_t pad[2];
};
static_assert(sizeof(SfItem) == 32, "SfItem layout");

// Workspace byte offsets (all 256-aligned).
struct WsLayout {
  int64_t plan, enum_chunk_tab, sf_items, peak_chunks, eblocks, crystal_order, bw_items, ab_items;
  int64_t enum_count, enum_prefix;
  int64_t atoms, atom_orig, runs, run_count, err_flag;
  int64_t bin_count, bin_start;
  int64_t skey, sidx, ent_key, ent_idx, ent_w, span_first, span_last;
  int64_t flags;
  int64_t cmax, pk_count, tmp_tt, tmp_i, tmp_mult, tmp_first;
  int64_t sort_items;  // the sort launch's crystal lists
  int64_t big_chunks, big_crystals, big_cnt, big_off, big_np, big_hist, big_boff, big_over;  // the many-block
                                                                                             // sort's tables
                                                                                             // and scratch
  int64_t scan_part;
  int64_t bw_w12, bw_ga, bw_gb, bw_dq, bw_part, bw_part6, bw_partf;  // bw_w12: (w1, w2) per reflection
  int64_t sf_deriv;  // kept (A, B, dA/ds^2, dB/ds^2) per reflection, or -1
  int64_t coeff_f;   // [n_species] CoeffF
  int64_t sf_items_bw;  // structure-factor items in the adjoint's launch order
  int64_t fam_ops;      // [n_crystals] FamOps
  int64_t rot;          // [N] AtomRot
  // row-recurrence structure factors: segment counts per entry, their scan,
  // segment starts, the entry count, the work items (or -1)
  int64_t seg_cnt, seg_index, seg_part, seg_start, n_entries, sf_items_rec, rec_of;
  int64_t total;
};

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Device address of the fixed scratch array (kNoallocBytes, 256-byte
// aligned) on the current device, looked up on the first call per device.
hipError_t noalloc_scratch(void **out);

// Two emission lines' peaks in one list per crystal (lines.hip).
struct LinePeaks {
  const double *two_theta, *intensity, *q;
  const int32_t *mult;
  const int64_t *first, *perm, *peak_offset;
  double weight;
};
struct LineOut {
  double *two_theta, *intensity, *scaled;
  int32_t *mult;
  double *d;
  int32_t *line;
  int64_t *source, *peak_offset;
};
void launch_combine_lines(int64_t n_c, const LinePeaks &p0, const LinePeaks *p1, const LineOut &out, hipStream_t s);

// Families of equivalent reflections per merged peak (rule 0: indices, 1: lattice).
void launch_peak_families(const HChunk *chunks, int64_t n_chunks, const FamOps *fam_ops, const int64_t *peak_offset,
                          const int64_t *first, const int32_t *mult, const int64_t *perm, const int16_t *h,
                          const int16_t *k, const int16_t *l, int rule, int32_t *n_fam, int32_t *fam_of,
                          int64_t *fam_label, int32_t *fam_mult, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);

// Exclusive scan of int32 in[0, n) into int64 out[0, n] (out[n] = total).
// If n_dev is non-null, only the first m = min(n, *n_dev) elements are
// scanned: out[0..m] is written (out[m] = total) and out[n] = total; the
// entries between are left as they were.  ``part`` needs scan_part_elems(n).
int64_t scan_part_elems(int64_t n);
void launch_scan_i32(const int32_t *in, int64_t n, const int64_t *n_dev, int64_t *out, int64_t *part,
                     hipStream_t s);


// ---- launch wrappers (defined in the .hip files) ---------------------------

struct BwItem {
  int32_t crystal, ablock, chunk, pad;
};
struct AbItem {
  int32_t crystal, ablock;
};

// Enumeration (count, scan, fill) and, in the same launches, the packing of
// the atoms into species runs for the structure-factor kernels.
// max_crystal_chunks: the most enumeration chunks of one crystal (INT64_MAX
// when a crystal has none); with few chunks the fill forms the offsets itself.
// max_crystal_atoms: the most atoms of one crystal (the packing of large
// crystals gets a launch of its own).
void launch_enumerate(const CrystalPlan *plan, int64_t n_c, const EnumChunk *chunks, int64_t n_chunks,
                      double lambda, int32_t *counts, int64_t *prefix, int64_t *scan_part, int16_t *h, int16_t *k,
                      int16_t *l, double *q, double *tt, double *lp, int64_t *refl_offset, int32_t n_species,
                      const double *frac, const int32_t *species, const double *occ, const double *bfac,
                      const double *coeff, CoeffF *coeff_f, AtomRec *atoms, AtomRot *rot, int32_t *orig,
                      SpeciesRun *runs, int32_t *run_count, int32_t *err, int64_t max_crystal_chunks,
                      int64_t max_crystal_atoms, hipStream_t s);
// Items: the first n_heavy take a block each (atoms split over its four
// wavefronts), the rest one wavefront each.  A non-null deriv_cache
// ([refl_cap] float4 under mixed precision, else double4) receives
// (A, B, dA/ds^2, dB/ds^2) of every evaluated reflection.
void launch_sf(bool mixed, bool friedel, const SfItem *items, int64_t n_items, int64_t n_heavy, const CrystalPlan *plan,
               const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l, const double *q,
               const double *lp, const AtomRec *atoms, const SpeciesRun *runs, const int32_t *run_count,
               const double *coeff, const CoeffF *coeff_f, void *A, void *B, double *I, void *deriv_cache,
               int rpt, hipStream_t s);

// Structure factors by the row recurrence (sfrec.hip): the segments of the
// current reflections are built first (kRecLen consecutive reflections of a
// row at most), then one lane per segment.
struct SfRecArgs {
  int64_t n_c;
  const SfItem *items;  // (crystal, tile of 64 segments), heavy items first
  int64_t n_items, n_heavy;
  const HChunk *eblocks;  // (crystal, block of kEntBlock evaluated reflections) at capacity
  int64_t n_eblocks;
  int64_t entry_cap;      // evaluated-reflection capacity of the batch
  const CrystalPlan *plan;
  const int64_t *refl_offset;
  const int16_t *h, *k, *l;
  const double *q, *lp;
  const AtomRec *atoms;
  const AtomRot *rot;
  const SpeciesRun *runs;
  const int32_t *run_count;
  const double *coeff;
  const CoeffF *coeff_f;
  int32_t *seg_cnt;       // [entry_cap]
  int64_t *seg_index;     // [entry_cap + 1]
  int64_t *seg_part;      // scan_part_elems(entry_cap)
  int32_t *seg_start;     // [entry_cap]
  int64_t *n_entries;     // [1]
  const int32_t *rec_of;  // [n_c] 1: the crystal takes the recurrence (only those get segments)
};
void launch_sf_rec(bool mixed, bool friedel, const SfRecArgs &a, void *A, void *B, double *I, void *deriv_cache,
                   hipStream_t s);

struct SortArgs {
  int64_t n_c;
  const CrystalPlan *plan;
  const int64_t *refl_offset;
  const double *tt;
  const int16_t *h, *k, *l;
  int32_t *bin_count;
  int64_t *bin_start;
  int64_t n_bins;
  double *skey;
  int32_t *sidx;
  const int32_t *order;  // [n_c] crystals by descending capacity
  int64_t n_small;       // leading entries of ``order`` with capacity above 2 kTinySort
  const int32_t *items;  // [n_small + n_c] the sort launch's crystals: those that may exceed
                         // 2 kTinySort reflections, then every crystal (four per block)
  int32_t friedel;       // write the evaluated-half entries below
  double *ent_key;       // [half capacity] 2theta of the evaluated half, sorted per crystal
  int32_t *ent_idx;      // its global reflection indices
  // crystals of capacity above kBigSort: their chunks and the crystals
  // themselves, per-chunk counters and their scans (3 each), per-crystal
  // peak counts and the bucket counters of the many-block sort
  const BigChunk *big_chunks;
  int64_t n_big_chunks;
  const BigChunk *big_crystals;
  int64_t n_big;
  int32_t big_nb_max;  // most buckets of a crystal
  int32_t *big_cnt;
  int64_t *big_off;
  int32_t *big_np;
  int32_t *big_hist;   // per (chunk, bucket) counts, then their column scans
  int64_t *big_boff;   // per (crystal, bucket) totals, then their offsets
  int64_t big_buckets; // buckets in all
  int2 *big_over;      // [big_buckets] large buckets listed by the wavefront sort, then their count (int32)
};
// Two more streams for independent work inside one call: the caller's stream
// records ``fork``, the side streams wait for it, run their parts and record
// ``join``/``join2``, which the caller's stream waits for before the call's
// next step (the pattern graph capture follows across streams).
// side == nullptr runs everything on the caller's stream.
struct Fork {
  hipStream_t side, side2;
  hipEvent_t fork, join, join2;
};

// Every sort of a call runs in one launch on the caller's stream.
void launch_sort(const SortArgs &a, hipStream_t s);

struct MergeArgs {
  SortArgs sort;
  int64_t n_c;
  double tol, thr;
  const double *inten;
  int32_t *flags;      // [refl_cap] peak starts of crystals sorted in global memory
  // each crystal's peaks staged at its reflection offset, with counts and maxima
  double *tmp_tt, *tmp_i;
  int32_t *tmp_mult;
  int64_t *tmp_first;
  int32_t *pk_count;   // [n_c]
  uint64_t *cmax;      // [n_c]
  const HChunk *peak_chunks;  // (crystal, chunk of kSortChunk peak slots), expected-filled first
  int64_t n_peak_chunks;
  // outputs
  double *pk_tt, *pk_i, *pk_y;
  int32_t *pk_mult;
  int64_t *pk_first, *perm, *peak_offset;
};
void launch_merge(const MergeArgs &a, hipStream_t s);

// Gaussian broadening over the sorted entries (evaluated reflections in
// 2theta order).  The forward also fills ent_w (double weights, or float
// weights in its first half under mixed precision) and the span tables;
// crystal_order lists the crystals heaviest first.  eblocks lists the
// (crystal, block of kEntBlock entries) units of the entry preparation and
// the adjoint, one workgroup each, the expected-filled ones first.
void launch_broaden_fwd(bool mixed, const HChunk *eblocks, int64_t n_eblocks, const CrystalPlan *plan,
                        const int32_t *crystal_order, int64_t n_c, bool friedel, const int64_t *refl_offset, const double *ent_key,
                        const int32_t *ent_idx, const double *inten, double t0, double dt, int64_t n, double sigma,
                        double window, int64_t span_cap, double *ent_w, int32_t *span_first, int32_t *span_last,
                        double *y, hipStream_t s);
void launch_broaden_adj(bool mixed, const HChunk *eblocks, int64_t n_eblocks, const CrystalPlan *plan,
                        bool friedel, const int64_t *refl_offset, const double *ent_key, const int32_t *ent_idx,
                        const double *dy, double t0, double dt, int64_t n, double sigma, double window, double2 *w12,
                        hipStream_t s);
void launch_sf_bw(bool mixed, bool friedel, const SfItem *items, int64_t n_items, int64_t n_heavy,
                  const CrystalPlan *plan,
                  const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l, const double *q,
                  const double *lp, double lambda, const AtomRec *atoms, const SpeciesRun *runs,
                  const int32_t *run_count, const double *coeff, const CoeffF *coeff_f, const void *deriv_cache,
                  const double2 *w12, double *ga, double *gb, double *dq, double *part6, double *part_fused,
                  int rpt, hipStream_t s);
size_t atom_bw_lds_bytes(bool mixed, int tile, int runs_cap);
void launch_atom_bw(bool mixed, bool friedel, const BwItem *items, int64_t n_items, const CrystalPlan *plan,
                    const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l,
                    const double *q, const double *ga, const double *gb, const AtomRec *atoms,
                    const SpeciesRun *runs, const int32_t *run_count, const double *coeff, const CoeffF *coeff_f,
                    int tile, int runs_cap, double *part, hipStream_t s);
// Preferred orientation (March-Dollase factor on I, in place; blocks from
// the peak chunk table) and noise on broadened patterns (in place).
void launch_march_dollase(const HChunk *chunks, int64_t n_chunks, const CrystalPlan *plan,
                          const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l,
                          const double *hp, const double *march_r, double *inten, hipStream_t s);
void launch_noise(int64_t total, uint64_t seed, double rel, double abs_, double *y, hipStream_t s);
// Broadened pattern with Caglioti widths over the sorted entries (the
// evaluated half under Friedel pairing, weight 2, else every reflection).
void launch_broaden_caglioti(bool mixed, const CrystalPlan *plan, int64_t n_c, const int64_t *refl_offset, bool friedel,
                             const double *ent_key, const int32_t *ent_idx, const double *inten, double t0,
                             double dt, int64_t n, double U, double V, double W, double eta, double window,
                             double *y, hipStream_t s);
// Atom gradients reduced over their partial rows and scattered to the
// caller's order, and, in the same launch, dL/d(lattice) of every crystal
// from its per-tile dL/dG* rows (written by launch_sf_bw).
void launch_bw_finish(const AbItem *items, int64_t n_ab, bool friedel, const CrystalPlan *plan, int64_t n_c,
                      const int64_t *refl_offset, const double *part, const double *part_fused, const int32_t *orig,
                      const double *part6, double *dfrac, double *dbfac, double *dlat, hipStream_t s);

}  // namespace xrd
