// C ABI of libxrd: validation, host planning, workspace layout and launches.
//
// Planning (the cell-preparation step) runs on the host once per batch: the
// inverse metric from the reciprocal-cell formulas, the search box of each
// crystal (|h| <= gmax a since h = g . a for a reciprocal vector g of length
// at most gmax = 2 sin(theta_max) / lambda), capacities, and the launch tables
// of every kernel.  The tables are sized at capacity so that every launch
// has a host-known grid; blocks whose work lies beyond a crystal's actual
// reflection count exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/xrd.h"
#include "xrd_internal.h"

using namespace xrd;

struct xrd_batch {
  xrd_batch_desc desc;
  std::vector<double> lattice, tmin, tmax;
  std::vector<int64_t> atom_offset;
  std::vector<CrystalPlan> plan;
  std::vector<EnumChunk> enum_chunks;  // enumeration chunks, crystal by crystal
  int64_t max_enum_chunks = 0;         // most chunks of one crystal (INT64_MAX if a crystal has none)
  int64_t max_atoms = 0;               // most atoms of one crystal
  std::vector<HChunk> peak_chunks;  // peak chunks of the merge (crystal, chunk)
  std::vector<HChunk> eblocks;  // entry blocks of the broadening (crystal, block of kEntBlock entries)
  std::vector<int32_t> crystal_order;  // crystals by descending reflection capacity
  std::vector<int32_t> sort_items;     // the sort launch's two crystal lists (n_small + n_crystals)
  std::vector<BigChunk> big_chunks, big_crystals;  // the many-block sort's chunks and crystals
  int64_t big_hist = 0, big_buckets = 0;           // its (chunk, bucket) counters and buckets in all
  int32_t big_nb_max = 0;
  std::vector<int32_t> sf_order;   // crystals by descending atom count
  std::vector<int32_t> sf_likely;  // per crystal: tiles its expected reflection count fills
  std::vector<SfItem> sf_items, sf_items_bw;  // launch orders of the forward sum and the adjoint
  std::vector<int32_t> rec_tiles, rec_likely;  // row recurrence: segment tiles per crystal (capacity, expected)
  std::vector<SfItem> sf_items_rec;            // launch order of the row-recurrence forward sum
  int64_t sf_heavy_rec = 0;
  bool rec = false;                            // the recurrence is available (sf_method not direct)
  int32_t rec_min_atoms = kRecMinAtoms;        // XRD_SF_AUTO: threshold of the per-crystal choice
  std::vector<int32_t> use_rec;                // per crystal: 1 if its forward sum takes the recurrence
  int64_t n_rec = 0;                           // crystals whose forward sum takes the recurrence
  std::vector<BwItem> bw_items;
  std::vector<AbItem> ab_items;
  std::vector<FamOps> fam_ops;  // lattice point operations per crystal
  int64_t n_atoms = 0, refl_cap = 0, half_cap = 0, n_bins = 0, run_cap = 0, part_rows = 0, partf_rows = 0;
  int64_t n_small = 0;    // crystals whose reflection capacity exceeds 2 kTinySort
  int64_t sf_heavy = 0, sf_heavy_bw = 0;  // leading items that take a block each
  int32_t split_fwd = kSplitFwd, split_bw = kSplitBw;
  int32_t rpt = kSfRptDefault;      // reflections per lane of the direct structure-factor kernels
  std::vector<double> expect_eval;  // per crystal: expected evaluated reflections
  int64_t grid_cap = 0;   // largest grid of a broadened-pattern call
  int64_t span_cap = 0;   // span-table entries per crystal: ceil(grid_cap / kSpanPts)
  int runs_cap_max = 1, bw_tile = 64;
  WsLayout ws{};
  WsLayout mws{};  // the merge's part only, packed (scratch of xrd_merge_peaks_noalloc)
  void *last_ws = nullptr;
  // the (2theta, hkl) order in a workspace is computed once per enumeration:
  // merge and broadening share it (host-side record of the call sequence, so
  // a captured graph replays the same decision)
  const void *sorted_ws = nullptr;
  const double *sorted_tt = nullptr;
  // derivatives kept by the last structure-factor call (keep_sf_derivs): the
  // workspace and reflection arrays they belong to; cleared by enumeration
  const void *deriv_ws = nullptr;
  const int16_t *deriv_h = nullptr;
  // side stream and events for work that runs beside the caller's stream
  // inside one call, created at first use on the then-current device
  int side_device = -1;
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_check(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return XRD_OK;
}

constexpr double kPi = 3.14159265358979323846;

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Inverse metric of a cell from the reciprocal-cell formulas; false if the
// cell is invalid (lengths <= 0, angles outside (0, 180), or flatness
// 1 - sum cos^2 + 2 prod cos below 1e-3).
bool reciprocal_metric(const double *lat, double gs[6]) {
  const double a = lat[0], b = lat[1], c = lat[2];
  if (!(a > 0) || !(b > 0) || !(c > 0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c)) return false;
  for (int i = 3; i < 6; ++i)
    if (!(lat[i] > 0.0 && lat[i] < 180.0)) return false;
  const double al = lat[3] * kPi / 180.0, be = lat[4] * kPi / 180.0, ga = lat[5] * kPi / 180.0;
  const double ca = std::cos(al), cb = std::cos(be), cg = std::cos(ga);
  const double sa = std::sin(al), sb = std::sin(be), sg = std::sin(ga);
  const double flat = 1.0 - ca * ca - cb * cb - cg * cg + 2.0 * ca * cb * cg;
  if (!(flat >= 1e-3)) return false;
  const double V = a * b * c * std::sqrt(flat);
  const double as = b * c * sa / V, bs = a * c * sb / V, cs = a * b * sg / V;
  const double cas = (cb * cg - ca) / (sb * sg);
  const double cbs = (ca * cg - cb) / (sa * sg);
  const double cgs = (ca * cb - cg) / (sa * sb);
  gs[0] = as * as;
  gs[1] = bs * bs;
  gs[2] = cs * cs;
  gs[3] = as * bs * cgs;
  gs[4] = as * cs * cbs;
  gs[5] = bs * cs * cas;
  return true;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Point operations of a lattice for the grouping of equivalent reflections:
// integer matrices M with entries in {-1, 0, 1}, det M = +-1 and
// M^T G* M = G* within 1e-6 of the largest diagonal entry of G*, acting as
// hkl -> M hkl.  Column j of such an M is a vector v with v^T G* v = G*_jj,
// so the search takes the candidate columns of each length first and then
// the triples whose cross terms match.  Also flags a hexagonal lattice
// (G*11 = G*22, G*13 = G*23 = 0, G*12 = G*11 / 2).
FamOps family_ops(const double gs[6]) {
  FamOps fo{};
  const double G[3][3] = {{gs[0], gs[3], gs[4]}, {gs[3], gs[1], gs[5]}, {gs[4], gs[5], gs[2]}};
  const double tol = 1e-6 * std::max(gs[0], std::max(gs[1], gs[2]));
  auto close = [&](double x, double y) { return std::fabs(x - y) <= tol; };
  auto form = [&](const int *u, const int *v) {
    double s = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int r = 0; r < 3; ++r) s += u[p] * G[p][r] * v[r];
    return s;
  };
  int vec[26][3], nv = 0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c)
        if (a || b || c) {
          vec[nv][0] = a;
          vec[nv][1] = b;
          vec[nv][2] = c;
          ++nv;
        }
  std::vector<int> cand[3];
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < nv; ++v)
      if (close(form(vec[v], vec[v]), G[j][j])) cand[j].push_back(v);
  for (int x : cand[0])
    for (int y : cand[1]) {
      if (!close(form(vec[x], vec[y]), G[0][1])) continue;
      for (int z : cand[2]) {
        if (!close(form(vec[x], vec[z]), G[0][2]) || !close(form(vec[y], vec[z]), G[1][2])) continue;
        const int *c0 = vec[x], *c1 = vec[y], *c2 = vec[z];  // columns of M
        const int det = c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1]) +
                        c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]);
        if (det != 1 && det != -1) continue;
        if (fo.n_ops == 48) continue;  // a lattice has at most 48; tolerance artefacts beyond are dropped
        uint32_t code = 0;
        for (int r = 0; r < 3; ++r) {
          code |= (uint32_t)(c0[r] + 1) << (6 * r);
          code |= (uint32_t)(c1[r] + 1) << (6 * r + 2);
          code |= (uint32_t)(c2[r] + 1) << (6 * r + 4);
        }
        fo.op[fo.n_ops++] = code;
      }
    }
  fo.hex = close(gs[0], gs[1]) && close(gs[4], 0.0) && close(gs[5], 0.0) && close(gs[3], 0.5 * gs[0]);
  return fo;
}

// Cut a crystal's half box into enumeration chunks: runs of consecutive rows
// (the lexicographic row order of the device enumeration: (0, 0), (0, k) for
// k = 1..K, then (h, k) for h = 1..H, k = -K..K) of at most kEnumRows rows,
// closed early when the next row would take the candidate count past
// kEnumCand.  A row's candidates are the l between the roots of the convex
// quadratic q(l) = qhi (one more on each side, clipped to the box), the same
// bounds the kernels use; here they only balance the chunks, so the host's
// rounding need not match the device's.  Appends to ``out``; returns the
// number of chunks.
int32_t enum_chunks_of(const CrystalPlan &P, int32_t c, std::vector<EnumChunk> *out) {
  const int64_t rows = (int64_t)P.H * (2 * P.K + 1) + P.K + 1;
  const double A = P.gs[2], lim = (double)P.L + 1.0;
  auto candidates = [&](int64_t rho) -> int64_t {
    int h, k;
    if (rho <= P.K) {
      h = 0;
      k = (int)rho;
    } else {
      const int64_t x = rho - (P.K + 1), nk = 2 * P.K + 1;
      h = 1 + (int)(x / nk);
      k = (int)(x % nk) - P.K;
    }
    const double B = 2.0 * (P.gs[4] * h + P.gs[5] * k);
    const double C = P.gs[0] * h * h + P.gs[1] * k * k + 2.0 * P.gs[3] * h * k;
    const double disc = B * B - 4.0 * A * (C - P.qhi * (1.0 + 1e-9));
    if (!(disc >= 0.0)) return 0;
    const double sq = std::sqrt(disc);
    const double r1 = std::fmin(std::fmax((-B - sq) / (2.0 * A), -lim), lim);
    const double r2 = std::fmin(std::fmax((-B + sq) / (2.0 * A), -lim), lim);
    const int64_t lo = std::max<int64_t>((h == 0 && k == 0) ? 1 : -P.L, (int64_t)std::floor(r1));
    const int64_t hi = std::min<int64_t>(P.L, (int64_t)std::ceil(r2));
    return std::max<int64_t>(0, hi - lo + 1);
  };
  int32_t n = 0;
  int64_t start = 0, cand = 0;
  for (int64_t rho = 0; rho < rows; ++rho) {
    const int64_t m = candidates(rho);
    if (rho > start && (rho - start == kEnumRows || cand + m > kEnumCand)) {
      out->push_back(EnumChunk{c, (int32_t)start, (int32_t)(rho - start), 0});
      ++n;
      start = rho;
      cand = 0;
    }
    cand += m;
  }
  out->push_back(EnumChunk{c, (int32_t)start, (int32_t)(rows - start), 0});
  return n + 1;
}

template <class T>
T *at(void *ws, int64_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

hipStream_t stream_of(const xrd_batch *b) { return static_cast<hipStream_t>(b->desc.stream); }

int check_ws(const xrd_batch *b, const void *ws) {
  if (!ws) return fail(XRD_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(XRD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  return XRD_OK;
}

int check_refl(const xrd_refl *r) {
  if (!r || !r->h || !r->k || !r->l || !r->q || !r->two_theta || !r->lp || !r->refl_offset)
    return fail(XRD_ERR_INVALID_ARG, "reflection arrays must be non-NULL");
  return XRD_OK;
}

// Structure-factor items in launch order for split threshold ``split``:
// the expected-filled tiles of the crystals with at least ``split`` atoms (a
// block per tile, atoms split over its wavefronts), then those of the other
// crystals (one wavefront per tile), then per crystal one item for its
// remaining capacity tiles, which a single wavefront walks in order: they
// mostly hold no reflection, and the few that do are complete on one
// wavefront.  Crystals come in descending atom count, so the heaviest work is
// dispatched first.
//
// The expected-filled items are placed so that a crystal's items run on one
// XCD (one L2 holds its atoms and reflections).  Workgroups reach the eight
// XCDs round-robin by block index, so block i runs on XCD i mod 8.  Crystals
// are spread over the XCDs by expected work (largest first, onto the least
// loaded); each XCD keeps a queue of its crystals in the order above.  The
// heavy items take a block each and the light ones four to a block, so slot
// i of the heavy part and the four slots of light block j draw the next tile
// of the queue of the XCD their block lands on; when that queue is empty,
// from the longest other one.  The items are written in that order directly.
//
// ``rec``: the row-recurrence tiles (64 segments each) instead of the direct
// kernel's (kSfTile reflections each).  ``forward``: only the crystals whose
// forward sum takes that method (the adjoint's table lists every crystal).
// Returns the number of block-per-tile items.
int64_t sf_table(const xrd_batch *b, int32_t split, std::vector<SfItem> *items, bool rec = false,
                 bool forward = false) {
  constexpr int kXcd = 8;
  items->clear();
  const int64_t nc = (int64_t)b->plan.size();
  auto listed = [&](int32_t c) { return !forward || b->use_rec.empty() || (b->use_rec[c] != 0) == rec; };
  auto tiles = [&](int32_t c) -> int32_t { return !listed(c) ? 0 : rec ? b->rec_tiles[c] : b->plan[c].n_tiles; };
  auto likely = [&](int32_t c) -> int32_t { return !listed(c) ? 0 : rec ? b->rec_likely[c] : b->sf_likely[c]; };
  auto item = [&](int32_t c, int32_t t, int32_t tail) {
    const CrystalPlan &P = b->plan[c];
    return SfItem{c, t, (int32_t)P.atom_begin, (int32_t)P.atom_end, (int32_t)P.run_begin, tail, {0, 0}};
  };
  auto heavy = [&](int32_t c) { return b->plan[c].atom_end - b->plan[c].atom_begin >= split; };
  // XCD of each crystal: by expected work, largest first, onto the least loaded
  std::vector<int8_t> xcd_of(nc, 0);
  {
    std::vector<std::pair<double, int32_t>> work;
    work.reserve(nc);
    for (int32_t c = 0; c < nc; ++c) {
      const CrystalPlan &P = b->plan[c];
      work.push_back({(double)likely(c) * (double)std::max<int64_t>(P.atom_end - P.atom_begin, 1), c});
    }
    std::stable_sort(work.begin(), work.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    double load[kXcd] = {};
    for (const auto &w : work) {
      int best = 0;
      for (int x = 1; x < kXcd; ++x)
        if (load[x] < load[best]) best = x;
      xcd_of[w.second] = (int8_t)best;
      load[best] += w.first;
    }
  }
  int64_t cap = 0;
  for (int32_t c = 0; c < nc; ++c) cap += likely(c) + (likely(c) < tiles(c) ? 1 : 0);
  items->reserve((size_t)cap);
  // one part (heavy or light): per-XCD queues of crystals with a cursor
  auto emit_part = [&](bool want_heavy, int per_block, int64_t first_block) {
    struct Queue {
      std::vector<int32_t> cr;
      size_t ci = 0;
      int32_t t = 0;
      int64_t left = 0;
    } q[kXcd];
    for (int32_t c : b->sf_order)
      if (heavy(c) == want_heavy && likely(c) > 0) {
        q[xcd_of[c]].cr.push_back(c);
        q[xcd_of[c]].left += likely(c);
      }
    int64_t remaining = 0;
    for (int x = 0; x < kXcd; ++x) remaining += q[x].left;
    for (int64_t blk = first_block; remaining > 0; ++blk) {
      const int x = (int)(blk % kXcd);
      for (int k = 0; k < per_block && remaining > 0; ++k) {
        int from = x;
        if (q[from].left == 0) {
          int64_t most = 0;
          for (int y = 0; y < kXcd; ++y)
            if (q[y].left > most) {
              most = q[y].left;
              from = y;
            }
        }
        Queue &Q = q[from];
        const int32_t c = Q.cr[Q.ci];
        items->push_back(item(c, Q.t, 0));
        if (++Q.t == likely(c)) {
          Q.t = 0;
          ++Q.ci;
        }
        --Q.left;
        --remaining;
      }
    }
  };
  emit_part(true, 1, 0);
  const int64_t n_heavy = (int64_t)items->size();
  emit_part(false, 4, n_heavy);  // four wavefronts to a light block
  for (int pass = 0; pass < 2; ++pass)
    for (int32_t c : b->sf_order)
      if (heavy(c) == (pass == 0) && likely(c) < tiles(c)) items->push_back(item(c, likely(c), 1));
  return n_heavy;
}

// XRD_SF_AUTO's per-crystal choice: the recurrence for crystals with at
// least rec_min_atoms atoms whose rows along l are long (the search box
// reaches |l| >= kRecMinRow, so rows of the shell hold a few segments);
// every crystal under XRD_SF_RECURRENCE, none under XRD_SF_DIRECT.  Then the
// forward tables of both methods.
void choose_methods(xrd_batch *b) {
  const int64_t nc = (int64_t)b->plan.size();
  b->use_rec.assign(nc, 0);
  b->n_rec = 0;
  for (int64_t c = 0; c < nc; ++c) {
    const CrystalPlan &P = b->plan[c];
    bool r = false;
    if (b->desc.sf_method == XRD_SF_RECURRENCE)
      r = true;
    else if (b->desc.sf_method == XRD_SF_AUTO)
      r = P.atom_end - P.atom_begin >= b->rec_min_atoms && P.L >= kRecMinRow;
    b->use_rec[c] = r ? 1 : 0;
    b->n_rec += r ? 1 : 0;
  }
  b->sf_heavy = sf_table(b, b->split_fwd, &b->sf_items, false, true);
  if (b->rec) b->sf_heavy_rec = sf_table(b, b->split_fwd, &b->sf_items_rec, true, true);
}

// Tile shape of the direct structure-factor kernels: ``rpt`` reflections per
// lane, tiles of 64 rpt reflections.  Places each crystal's tiles, its rows
// of the per-tile tables (packed from the start of the workspace's arrays,
// which are sized for the finest shape) and its expected-filled tile count.
// The work tables (choose_methods, the adjoint's sf_table) are built after.
void set_tiles(xrd_batch *b, int32_t rpt) {
  b->rpt = rpt;
  const int64_t tile = 64 * (int64_t)rpt;
  const bool friedel = b->desc.friedel != 0;
  const int64_t nc = (int64_t)b->plan.size();
  b->sf_likely.resize(nc);
  int64_t tb = 0, pf = 0;
  for (int64_t c = 0; c < nc; ++c) {
    CrystalPlan &P = b->plan[c];
    const int64_t evalcap = friedel ? P.half_box : 2 * P.half_box;
    P.sf_tile = (int16_t)tile;
    P.n_tiles = (int32_t)ceil_div(evalcap, tile);
    P.tile_begin = (int32_t)tb;
    tb += P.n_tiles;
    if (P.fused) {
      P.pf_begin = pf;
      pf += (int64_t)P.n_tiles * (P.atom_end - P.atom_begin);
    }
    b->sf_likely[c] = (int32_t)std::min<double>((double)P.n_tiles, std::ceil((b->expect_eval[c] + tile) / tile));
  }
}

}  // namespace

// Host-side sizes shared with the kernels' launch code.
int64_t xrd::scan_part_elems(int64_t n) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  return (nb > 0 ? nb : 1) + 1;
}

// LDS of the atom-major adjoint block: the staged reflection tile (h, k, l in
// double; s^2, gA, gB and the species' scattering factors in the working
// precision) and the species coefficients, or the slice reduction (one
// double4 per thread) that reuses the space, whichever is larger.
size_t xrd::atom_bw_lds_bytes(bool mixed, int tile, int runs_cap) {
  const size_t rs = mixed ? sizeof(float) : sizeof(double);
  const size_t tiles = (size_t)tile * 3 * sizeof(double) + (size_t)tile * 3 * rs + (size_t)tile * runs_cap * rs +
                       (size_t)runs_cap * 9 * rs;
  const size_t red = (size_t)kSfThreads * 4 * sizeof(double);
  return tiles > red ? tiles : red;
}

extern "C" {

const char *xrd_last_error(void) { return g_err.c_str(); }

const char *xrd_version(void) { return "xrd-gfx950 1.0"; }

int xrd_batch_create(const xrd_batch_desc *d, xrd_batch **out) {
  if (!out) return fail(XRD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return fail(XRD_ERR_INVALID_ARG, "desc is NULL");
  const int64_t nc = d->n_crystals;
  if (nc < 0) return fail(XRD_ERR_INVALID_ARG, "n_crystals < 0");
  if (nc > (int64_t)1 << 30) return fail(XRD_ERR_CAPACITY, "n_crystals too large");
  if (d->n_species < 1) return fail(XRD_ERR_INVALID_ARG, "n_species < 1");
  if (d->n_species > 8192) return fail(XRD_ERR_CAPACITY, "n_species > 8192");
  if (d->precision != XRD_FP64 && d->precision != XRD_MIXED) return fail(XRD_ERR_INVALID_ARG, "unknown precision");
  if (d->friedel != 0 && d->friedel != 1) return fail(XRD_ERR_INVALID_ARG, "friedel must be 0 or 1");
  if (!(d->wavelength > 0.0) || !std::isfinite(d->wavelength)) return fail(XRD_ERR_INVALID_ARG, "wavelength must be > 0");
  if (!(d->merge_tol > 0.0) || !std::isfinite(d->merge_tol)) return fail(XRD_ERR_INVALID_ARG, "merge_tol must be > 0");
  if (!(d->rel_threshold >= 0.0) || !std::isfinite(d->rel_threshold))
    return fail(XRD_ERR_INVALID_ARG, "rel_threshold must be >= 0");
  if (d->grid_capacity < 0) return fail(XRD_ERR_INVALID_ARG, "grid_capacity < 0");
  if (d->keep_sf_derivs != 0 && d->keep_sf_derivs != 1)
    return fail(XRD_ERR_INVALID_ARG, "keep_sf_derivs must be 0 or 1");
  if (d->sf_rpt != 0 && d->sf_rpt != 1 && d->sf_rpt != 2 && d->sf_rpt != 4)
    return fail(XRD_ERR_INVALID_ARG, "sf_rpt must be 0, 1, 2 or 4");
  if (d->sf_method != XRD_SF_DIRECT && d->sf_method != XRD_SF_RECURRENCE && d->sf_method != XRD_SF_AUTO)
    return fail(XRD_ERR_INVALID_ARG, "unknown sf_method");
  if (d->forward_only != 0 && d->forward_only != 1) return fail(XRD_ERR_INVALID_ARG, "forward_only must be 0 or 1");
  if (nc > 0 && (!d->lattice || !d->atom_offset || !d->two_theta_min || !d->two_theta_max))
    return fail(XRD_ERR_INVALID_ARG, "host arrays must be non-NULL");
  if (!d->sf_coeff) return fail(XRD_ERR_INVALID_ARG, "sf_coeff is NULL");
  if (nc > 0 && d->atom_offset[0] != 0) return fail(XRD_ERR_INVALID_ARG, "atom_offset[0] must be 0");
  for (int64_t c = 0; c < nc; ++c)
    if (d->atom_offset[c + 1] < d->atom_offset[c]) return fail(XRD_ERR_INVALID_ARG, "atom_offset must be non-decreasing");
  const int64_t n_atoms = nc > 0 ? d->atom_offset[nc] : 0;
  if (n_atoms >= ((int64_t)1 << 31)) return fail(XRD_ERR_CAPACITY, "more than 2^31 atoms");
  if (n_atoms > 0 && (!d->frac || !d->species || !d->occ || !d->bfac))
    return fail(XRD_ERR_INVALID_ARG, "atom arrays must be non-NULL");
  for (int64_t c = 0; c < nc; ++c) {
    const double lo = d->two_theta_min[c], hi = d->two_theta_max[c];
    if (!(lo >= 0.0) || !(hi > lo) || !(hi < 180.0))
      return fail(XRD_ERR_INVALID_ARG, "crystal " + std::to_string(c) + ": need 0 <= two_theta_min < two_theta_max < 180");
  }

  xrd_batch *b = new (std::nothrow) xrd_batch();
  if (!b) return fail(XRD_ERR_INVALID_ARG, "out of host memory");
  b->desc = *d;
  b->lattice.assign(d->lattice, d->lattice + 6 * nc);
  b->atom_offset.assign(d->atom_offset, d->atom_offset + nc + 1);
  b->tmin.assign(d->two_theta_min, d->two_theta_min + nc);
  b->tmax.assign(d->two_theta_max, d->two_theta_max + nc);
  b->desc.lattice = b->lattice.data();
  b->desc.atom_offset = b->atom_offset.data();
  b->desc.two_theta_min = b->tmin.data();
  b->desc.two_theta_max = b->tmax.data();
  b->n_atoms = n_atoms;
  b->plan.resize(nc);
  b->fam_ops.resize(nc);

  const bool friedel = d->friedel != 0;
  const double lam = d->wavelength;
  int64_t ec = 0, sc = 0, hc = 0, bins = 0, runs = 0, parts = 0, pfused = 0, refl = 0, tiles_total = 0;
  int runs_cap_max = 1;
  for (int64_t c = 0; c < nc; ++c) {
    CrystalPlan &P = b->plan[c];
    std::memset(&P, 0, sizeof(P));
    const double *lat = b->lattice.data() + 6 * c;
    if (!reciprocal_metric(lat, P.gs)) {
      delete b;
      return fail(XRD_ERR_INVALID_CELL, "crystal " + std::to_string(c) + ": invalid cell");
    }
    for (int i = 0; i < 6; ++i) P.lat[i] = lat[i];
    P.tmin = b->tmin[c];
    P.tmax = b->tmax[c];
    const double gmax = 2.0 * std::sin(0.5 * P.tmax * kPi / 180.0) / lam;
    const double gmin = 2.0 * std::sin(0.5 * P.tmin * kPi / 180.0) / lam;
    P.qhi = gmax * gmax * (1.0 + 1e-9);
    P.qlo = gmin * gmin * (1.0 - 1e-9);
    const double bh = std::floor(gmax * lat[0] * (1.0 + 1e-9));
    const double bk = std::floor(gmax * lat[1] * (1.0 + 1e-9));
    const double bl = std::floor(gmax * lat[2] * (1.0 + 1e-9));
    if (bh > 16000 || bk > 16000 || bl > 16000) {
      delete b;
      return fail(XRD_ERR_CAPACITY, "crystal " + std::to_string(c) + ": search box exceeds 16000 in an index");
    }
    P.H = (int32_t)bh;
    P.K = (int32_t)bk;
    P.L = (int32_t)bl;
    const int64_t box = (2 * (int64_t)P.H + 1) * (2 * (int64_t)P.K + 1) * (2 * (int64_t)P.L + 1);
    if (box >= ((int64_t)1 << 31)) {
      delete b;
      return fail(XRD_ERR_CAPACITY, "crystal " + std::to_string(c) + ": search box exceeds 2^31 points");
    }
    P.half_box = (box - 1) / 2;
    refl += 2 * P.half_box;
    if (P.half_box > kTinySort) ++b->n_small;
    if (refl >= ((int64_t)1 << 31) - 1) {
      delete b;
      return fail(XRD_ERR_CAPACITY, "reflection capacity exceeds 2^31; split the batch");
    }
    P.sort_chunk_begin = sc;
    // at least one, so that every crystal has a block of the peak move (which
    // also writes its peak offset)
    P.sort_chunks = (int32_t)std::max<int64_t>(1, ceil_div(2 * P.half_box, kSortChunk));
    sc += P.sort_chunks;
    // (the many-block sort of the largest crystals uses buckets of its own)
    P.n_bins = 2 * P.half_box > kBigSort ? 1 : (int32_t)std::max<int64_t>(1, 2 * P.half_box / kBinDiv);
    P.bin_begin = bins;
    P.bin_scale = (double)P.n_bins / (P.tmax - P.tmin);
    bins += P.n_bins;
    P.atom_begin = b->atom_offset[c];
    P.atom_end = b->atom_offset[c + 1];
    const int64_t na = P.atom_end - P.atom_begin;
    const int64_t rc = std::min<int64_t>(d->n_species, na);
    P.run_begin = runs;
    runs += rc;
    runs_cap_max = (int)std::max<int64_t>(runs_cap_max, rc);
    const int64_t evalcap = friedel ? P.half_box : 2 * P.half_box;
    // at least one chunk, so that every crystal gets its lattice gradient
    P.n_hchunks = (int32_t)std::max<int64_t>(1, ceil_div(evalcap, kHalfChunk));
    P.hchunk_begin = hc;
    hc += P.n_hchunks;
    // structure-factor tiles at the finest shape, for which the per-tile
    // tables of the workspace are sized (set_tiles places them for the
    // batch's shape)
    const int64_t fine_tiles = ceil_div(evalcap, 64 * kSfRptMin);
    tiles_total += fine_tiles;
    P.fused = na <= kFusedMaxAtoms ? 1 : 0;
    b->max_atoms = std::max<int64_t>(b->max_atoms, na);
    if (P.fused) {
      pfused += fine_tiles * na;
    } else {
      P.part_begin = parts;
      parts += (int64_t)P.n_hchunks * na;
    }
  }
  // the enumeration chunks (a pass over every row of a crystal's search box)
  // and the lattice operations, crystal by crystal on up to 16 host threads,
  // then concatenated in crystal order
  {
    std::vector<std::vector<EnumChunk>> chunks_of(nc);
    const int64_t nt = std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16, (nc + 63) / 64}));
    auto work = [&](int64_t t) {
      for (int64_t c = t; c < nc; c += nt) {
        enum_chunks_of(b->plan[c], (int32_t)c, &chunks_of[c]);
        b->fam_ops[c] = family_ops(b->plan[c].gs);
      }
    };
    std::vector<std::thread> pool;
    int64_t started = 1;
    try {
      for (; started < nt; ++started) pool.emplace_back(work, started);
    } catch (...) {
      // no more threads: the shares left over run here
    }
    work(0);
    for (auto &th : pool) th.join();
    for (int64_t t = started; t < nt; ++t) work(t);
    for (int64_t c = 0; c < nc; ++c) {
      CrystalPlan &P = b->plan[c];
      P.enum_chunk_begin = ec;
      P.enum_chunks = (int32_t)chunks_of[c].size();
      b->max_enum_chunks = P.enum_chunks == 0 ? INT64_MAX : std::max<int64_t>(b->max_enum_chunks, P.enum_chunks);
      ec += P.enum_chunks;
      b->enum_chunks.insert(b->enum_chunks.end(), chunks_of[c].begin(), chunks_of[c].end());
    }
  }
  b->refl_cap = refl;
  b->half_cap = refl / 2;
  b->grid_cap = d->grid_capacity > 0 ? d->grid_capacity : 16384;
  b->span_cap = ceil_div(b->grid_cap, kSpanPts);
  b->n_bins = bins;
  b->run_cap = runs;
  b->part_rows = parts;
  b->partf_rows = pfused;
  b->runs_cap_max = runs_cap_max;
  const bool mixed = d->precision == XRD_MIXED;
  int tile = 256;
  while (tile > 8 && atom_bw_lds_bytes(mixed, tile, runs_cap_max) > 48 * 1024) tile /= 2;
  b->bw_tile = tile;
  if (atom_bw_lds_bytes(mixed, tile, runs_cap_max) > 48 * 1024) {
    delete b;
    return fail(XRD_ERR_CAPACITY, "too many species per crystal for the adjoint's LDS tile");
  }

  // launch tables
  // Capacities come from the search box; the reflections a crystal actually
  // has are close to the lattice points of its spherical shell, (4 pi / 3)
  // (g_max^3 - g_min^3) V (both halves).  The launch tables list first the
  // work units this count (plus 5%) fills and then the rest, which mostly
  // find nothing to do and end at once.
  std::vector<double> expect_eval(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const CrystalPlan &P = b->plan[c];
    const double *lat = b->lattice.data() + 6 * c;
    const double r = kPi / 180.0, ca = std::cos(lat[3] * r), cb = std::cos(lat[4] * r), cg = std::cos(lat[5] * r);
    const double vol =
        lat[0] * lat[1] * lat[2] * std::sqrt(std::max(0.0, 1 - ca * ca - cb * cb - cg * cg + 2 * ca * cb * cg));
    const double ghi = std::sqrt(P.qhi), glo = std::sqrt(P.qlo);
    const double shell = 4.0 * kPi / 3.0 * (ghi * ghi * ghi - glo * glo * glo) * vol;
    expect_eval[c] = (friedel ? 0.5 : 1.0) * shell * 1.05;
  }
  auto likely_units = [&](int64_t c, int64_t unit, int64_t cap) {
    return (int32_t)std::min<double>((double)cap, std::ceil((expect_eval[c] + unit) / unit));
  };
  // gather order: crystals by descending capacity (their broadening cost)
  b->crystal_order.resize(nc);
  for (int64_t c = 0; c < nc; ++c) b->crystal_order[c] = (int32_t)c;
  std::stable_sort(b->crystal_order.begin(), b->crystal_order.end(),
                   [&](int32_t x, int32_t y) { return b->plan[x].half_box > b->plan[y].half_box; });
  // sort launch lists, each expected-heaviest first: the crystals whose
  // capacity exceeds 2 kTinySort reflections (a block each), then every
  // crystal for the blocks that sort four small ones at a time, those
  // expected at or below 2 kTinySort first (a group finds the others taken
  // by their own block and idles; four such groups end their block at once)
  {
    const double fr = friedel ? 2.0 / 1.05 : 1.0 / 1.05;  // expected reflections per expect_eval
    std::vector<int32_t> by_expect(nc);
    for (int64_t c = 0; c < nc; ++c) by_expect[c] = (int32_t)c;
    std::stable_sort(by_expect.begin(), by_expect.end(),
                     [&](int32_t x, int32_t y) { return expect_eval[x] > expect_eval[y]; });
    b->sort_items.clear();
    b->sort_items.reserve(b->n_small + nc);
    for (int32_t c : by_expect)
      if (b->plan[c].half_box > kTinySort) b->sort_items.push_back(c);
    for (int32_t c : by_expect)
      if (fr * expect_eval[c] <= 2 * kTinySort) b->sort_items.push_back(c);
    for (int32_t c : by_expect)
      if (fr * expect_eval[c] > 2 * kTinySort) b->sort_items.push_back(c);
    // crystals of capacity above kBigSort, expected-heaviest first, with
    // every chunk of their capacity
    b->big_chunks.clear();
    b->big_crystals.clear();
    b->big_hist = b->big_buckets = 0;
    b->big_nb_max = 0;
    int32_t first = 0;
    for (int32_t c : by_expect) {
      const int64_t cap = 2 * b->plan[c].half_box;
      if (cap <= kBigSort) continue;
      const int32_t n = (int32_t)ceil_div(cap, kBigChunk);
      // buckets of 128-256 capacity slots (about 70-130 reflections), a
      // power of two in [64, kBigBucketsMax]
      int32_t nb = 64;
      while (nb < kBigBucketsMax && (int64_t)nb * 256 < cap) nb *= 2;
      const BigChunk bc{c, 0, first, n, nb, 0, b->big_hist, b->big_buckets};
      b->big_crystals.push_back(bc);
      for (int32_t k = 0; k < n; ++k) {
        BigChunk ck = bc;
        ck.chunk = k;
        b->big_chunks.push_back(ck);
      }
      first += n;
      b->big_hist += (int64_t)n * nb;
      b->big_buckets += nb;
      b->big_nb_max = std::max(b->big_nb_max, nb);
    }
  }
  // peak chunks: a crystal's peaks are about half its reflections (mates share 2theta)
  {
    std::vector<int32_t> split(nc);
    for (int64_t c = 0; c < nc; ++c) {
      const double refl = expect_eval[c] * (friedel ? 2.0 : 1.0);
      split[c] = (int32_t)std::min<double>(b->plan[c].sort_chunks, std::ceil((0.5 * refl + kSortChunk) / kSortChunk));
      for (int32_t i = 0; i < split[c]; ++i) b->peak_chunks.push_back(HChunk{(int32_t)c, i});
    }
    for (int64_t c = 0; c < nc; ++c)
      for (int32_t i = split[c]; i < b->plan[c].sort_chunks; ++i) b->peak_chunks.push_back(HChunk{(int32_t)c, i});
  }
  // entry blocks, heaviest crystals first, the expected-filled blocks of
  // every crystal before all the rest (which mostly end at once), so that
  // the blocks with work are the first to find a workgroup slot
  {
    std::vector<int32_t> split(nc), n_eb(nc);
    for (int32_t c : b->crystal_order) {
      const CrystalPlan &P = b->plan[c];
      n_eb[c] = (int32_t)std::max<int64_t>(1, ceil_div(friedel ? P.half_box : 2 * P.half_box, kEntBlock));
      split[c] = likely_units(c, kEntBlock, n_eb[c]);
      for (int32_t i = 0; i < split[c]; ++i) b->eblocks.push_back(HChunk{c, i});
    }
    for (int32_t c : b->crystal_order)
      for (int32_t i = split[c]; i < n_eb[c]; ++i) b->eblocks.push_back(HChunk{c, i});
  }
  // structure-factor items: crystals in descending atom count (the cost of
  // one item), so the heaviest work is dispatched first
  b->sf_order.resize(nc);
  for (int64_t c = 0; c < nc; ++c) b->sf_order[c] = (int32_t)c;
  b->expect_eval = expect_eval;
  set_tiles(b, d->sf_rpt == 0 ? kSfRptDefault : d->sf_rpt);
  std::stable_sort(b->sf_order.begin(), b->sf_order.end(), [&](int32_t x, int32_t y) {
    return (b->atom_offset[x + 1] - b->atom_offset[x]) > (b->atom_offset[y + 1] - b->atom_offset[y]);
  });
  const bool adjoint = d->forward_only == 0;
  for (int32_t c : b->sf_order) {
    if (!adjoint) break;
    const CrystalPlan &P = b->plan[c];
    const int64_t na = P.atom_end - P.atom_begin;
    const int64_t ab = ceil_div(na, kAtomBlock);
    for (int64_t a = 0; a < ab; ++a) {
      b->ab_items.push_back(AbItem{(int32_t)c, (int32_t)a});
      if (!P.fused)
        for (int32_t k = 0; k < P.n_hchunks; ++k) b->bw_items.push_back(BwItem{(int32_t)c, (int32_t)a, k, 0});
    }
  }
  if (adjoint) b->sf_heavy_bw = sf_table(b, b->split_bw, &b->sf_items_bw);
  b->rec = d->sf_method != XRD_SF_DIRECT;
  if (b->rec) {
    // segments: at most one per evaluated reflection (capacity); expected
    // about one per kRecLen - 2 reflections (runs end mid-segment)
    b->rec_tiles.resize(nc);
    b->rec_likely.resize(nc);
    for (int64_t c = 0; c < nc; ++c) {
      const CrystalPlan &P = b->plan[c];
      const int64_t ecap = friedel ? P.half_box : 2 * P.half_box;
      b->rec_tiles[c] = (int32_t)ceil_div(ecap, 64);
      b->rec_likely[c] = (int32_t)std::min<double>((double)b->rec_tiles[c],
                                                   std::ceil((expect_eval[c] / (kRecLen - 2) + 64) / 64));
    }
  }
  choose_methods(b);
  if (tiles_total + nc >= ((int64_t)1 << 31) || (int64_t)b->bw_items.size() >= ((int64_t)1 << 31) ||
      (int64_t)b->sf_items_rec.size() >= ((int64_t)1 << 31)) {
    delete b;
    return fail(XRD_ERR_CAPACITY, "launch tables exceed 2^31 entries");
  }

  // workspace layout
  WsLayout &L = b->ws;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t r = o;
    o = align256(o + std::max<int64_t>(bytes, 8));
    return r;
  };
  const int64_t rc = b->refl_cap;
  L.plan = take((int64_t)sizeof(CrystalPlan) * nc);
  L.enum_chunk_tab = take((int64_t)sizeof(EnumChunk) * ec);
  // every crystal's tiles and one tail item each, at the finest tile shape
  // (the shape, split and methods may change)
  L.sf_items = take((int64_t)sizeof(SfItem) * (tiles_total + nc));
  L.sf_items_bw = take(adjoint ? (int64_t)sizeof(SfItem) * (tiles_total + nc) : 0);
  L.peak_chunks = take((int64_t)sizeof(HChunk) * sc);
  L.eblocks = take((int64_t)sizeof(HChunk) * (int64_t)b->eblocks.size());
  L.crystal_order = take(4 * nc);
  L.bw_items = take((int64_t)sizeof(BwItem) * (int64_t)b->bw_items.size());
  L.ab_items = take((int64_t)sizeof(AbItem) * (int64_t)b->ab_items.size());
  L.enum_count = take(4 * ec);
  L.enum_prefix = take(8 * (ec + 1));
  L.atoms = take((int64_t)sizeof(AtomRec) * n_atoms);
  L.atom_orig = take(4 * n_atoms);
  L.runs = take((int64_t)sizeof(SpeciesRun) * runs);
  L.run_count = take(4 * nc);
  L.err_flag = take(4);
  L.bin_count = take(4 * bins);
  L.bin_start = take(8 * (bins + 1));
  L.skey = take(8 * rc);
  L.sidx = take(4 * rc);
  // entries (evaluated reflections in 2theta order): their own arrays under
  // Friedel pairing, the full sorted list otherwise
  L.ent_key = friedel ? take(8 * b->half_cap) : L.skey;
  L.ent_idx = friedel ? take(4 * b->half_cap) : L.sidx;
  L.ent_w = take(8 * (friedel ? b->half_cap : rc));
  L.span_first = take(4 * nc * b->span_cap);
  L.span_last = take(4 * nc * b->span_cap);
  L.flags = take(4 * rc);
  L.cmax = take(8 * nc);
  L.pk_count = take(4 * nc);
  L.tmp_tt = take(8 * rc);
  L.tmp_i = take(8 * rc);
  L.tmp_mult = take(4 * rc);
  L.tmp_first = take(8 * rc);
  L.sort_items = take(4 * (b->n_small + nc));
  const int64_t nbc = (int64_t)b->big_chunks.size(), nbig = (int64_t)b->big_crystals.size();
  L.big_chunks = take((int64_t)sizeof(BigChunk) * nbc);
  L.big_crystals = take((int64_t)sizeof(BigChunk) * nbig);
  L.big_cnt = take(4 * 3 * nbc);
  L.big_off = take(8 * 3 * nbc);
  L.big_np = take(4 * nc);
  L.big_hist = take(4 * b->big_hist);
  L.big_boff = take(8 * b->big_buckets);
  L.big_over = take(8 * b->big_buckets + 8);
  int64_t scan_n = std::max<int64_t>(std::max<int64_t>(ec, bins), rc);
  L.scan_part = take(8 * scan_part_elems(scan_n));
  L.bw_w12 = L.bw_ga = L.bw_gb = L.bw_dq = L.bw_part = L.bw_partf = L.bw_part6 = -1;
  if (adjoint) {
    L.bw_w12 = take(16 * rc);
    L.bw_ga = take(8 * rc);
    L.bw_gb = take(8 * rc);
    L.bw_dq = take(8 * rc);
    L.bw_part = take(32 * parts);
    L.bw_partf = take(32 * pfused);
    L.bw_part6 = take(48 * tiles_total);
  }
  L.sf_deriv = d->keep_sf_derivs ? take((d->precision == XRD_MIXED ? 16 : 32) * rc) : -1;
  L.coeff_f = take((int64_t)sizeof(CoeffF) * d->n_species);
  L.fam_ops = take((int64_t)sizeof(FamOps) * nc);
  L.rot = take((int64_t)sizeof(AtomRot) * n_atoms);
  L.seg_cnt = L.seg_index = L.seg_part = L.seg_start = L.n_entries = L.sf_items_rec = L.rec_of = -1;
  if (b->rec) {
    const int64_t ecap = friedel ? b->half_cap : rc;
    L.seg_cnt = take(4 * ecap);
    L.seg_index = take(8 * (ecap + 1));
    L.seg_part = take(8 * scan_part_elems(ecap));
    L.seg_start = take(4 * ecap);
    L.n_entries = take(8);
    int64_t rt = 0;
    for (int32_t t : b->rec_tiles) rt += t;
    L.sf_items_rec = take((int64_t)sizeof(SfItem) * rt);
    L.rec_of = take(4 * nc);
  }
  L.total = o;
  // the merge's own tables and scratch, packed on their own for the
  // allocation-free merge (fields it does not use stay 0)
  {
    WsLayout &M = b->mws;
    o = 0;
    M.plan = take((int64_t)sizeof(CrystalPlan) * nc);
    M.peak_chunks = take((int64_t)sizeof(HChunk) * sc);
    M.crystal_order = take(4 * nc);
    M.bin_count = take(4 * bins);
    M.bin_start = take(8 * (bins + 1));
    M.skey = take(8 * rc);
    M.sidx = take(4 * rc);
    M.ent_key = friedel ? take(8 * b->half_cap) : M.skey;
    M.ent_idx = friedel ? take(4 * b->half_cap) : M.sidx;
    M.flags = take(4 * rc);
    M.cmax = take(8 * nc);
    M.pk_count = take(4 * nc);
    M.tmp_tt = take(8 * rc);
    M.tmp_i = take(8 * rc);
    M.tmp_mult = take(4 * rc);
    M.tmp_first = take(8 * rc);
    M.sort_items = take(4 * (b->n_small + nc));
    M.big_chunks = take((int64_t)sizeof(BigChunk) * nbc);
    M.big_crystals = take((int64_t)sizeof(BigChunk) * nbig);
    M.big_cnt = take(4 * 3 * nbc);
    M.big_off = take(8 * 3 * nbc);
    M.big_np = take(4 * nc);
    M.big_hist = take(4 * b->big_hist);
    M.big_boff = take(8 * b->big_buckets);
    M.big_over = take(8 * b->big_buckets + 8);
    M.total = o;
  }
  *out = b;
  g_err.clear();
  return XRD_OK;
}

int xrd_batch_sizes(const xrd_batch *b, xrd_sizes *out) {
  if (!b || !out) return fail(XRD_ERR_INVALID_ARG, "NULL argument");
  out->n_crystals = b->desc.n_crystals;
  out->n_atoms = b->n_atoms;
  out->refl_capacity = b->refl_cap;
  out->peak_capacity = b->refl_cap;
  out->workspace_bytes = b->ws.total;
  out->half_capacity = b->half_cap;
  out->noalloc_merge_bytes = b->mws.total;
  return XRD_OK;
}

int xrd_batch_set_lattice(xrd_batch *b, const double *lattice, void *ws) {
  if (!b || !lattice) return fail(XRD_ERR_INVALID_ARG, "batch or lattice is NULL");
  if (int e = check_ws(b, ws)) return e;
  const int64_t nc = b->desc.n_crystals;
  const double lam = b->desc.wavelength;
  std::vector<double> gs(6 * nc);
  for (int64_t c = 0; c < nc; ++c) {
    const double *lat = lattice + 6 * c;
    if (!reciprocal_metric(lat, gs.data() + 6 * c))
      return fail(XRD_ERR_INVALID_CELL, "crystal " + std::to_string(c) + ": invalid cell");
    const CrystalPlan &P = b->plan[c];
    const double gmax = 2.0 * std::sin(0.5 * P.tmax * kPi / 180.0) / lam;
    if (std::floor(gmax * lat[0] * (1.0 + 1e-9)) > P.H || std::floor(gmax * lat[1] * (1.0 + 1e-9)) > P.K ||
        std::floor(gmax * lat[2] * (1.0 + 1e-9)) > P.L)
      return fail(XRD_ERR_CAPACITY, "crystal " + std::to_string(c) + ": the new cell needs a larger search box");
  }
  // every crystal fits its box: take the new metric (the boxes, capacities
  // and launch tables stay; the kernels bound each row from the metric)
  for (int64_t c = 0; c < nc; ++c) {
    CrystalPlan &P = b->plan[c];
    for (int i = 0; i < 6; ++i) {
      P.gs[i] = gs[6 * c + i];
      P.lat[i] = lattice[6 * c + i];
      b->lattice[6 * c + i] = lattice[6 * c + i];
    }
    b->fam_ops[c] = family_ops(P.gs);
  }
  hipStream_t s = stream_of(b);
  const WsLayout &L = b->ws;
  hipError_t e = hipMemcpyAsync(at<char>(ws, L.plan), b->plan.data(), sizeof(CrystalPlan) * nc, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, L.fam_ops), b->fam_ops.data(), sizeof(FamOps) * nc, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("set_lattice: ") + hipGetErrorString(e));
  b->sorted_ws = nullptr;
  b->sorted_tt = nullptr;
  b->deriv_ws = nullptr;
  b->deriv_h = nullptr;
  return XRD_OK;
}

int xrd_batch_set_stream(xrd_batch *b, void *stream) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  b->desc.stream = stream;
  return XRD_OK;
}

int xrd_batch_upload(xrd_batch *b, void *ws) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  hipStream_t s = stream_of(b);
  const WsLayout &L = b->ws;
  auto up = [&](int64_t off, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(at<char>(ws, off), src, bytes, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(L.plan, b->plan.data(), sizeof(CrystalPlan) * b->plan.size());
  if (e == hipSuccess) e = up(L.enum_chunk_tab, b->enum_chunks.data(), sizeof(EnumChunk) * b->enum_chunks.size());
  if (e == hipSuccess) e = up(L.sf_items, b->sf_items.data(), sizeof(SfItem) * b->sf_items.size());
  if (e == hipSuccess) e = up(L.sf_items_bw, b->sf_items_bw.data(), sizeof(SfItem) * b->sf_items_bw.size());
  if (e == hipSuccess) e = up(L.peak_chunks, b->peak_chunks.data(), sizeof(HChunk) * b->peak_chunks.size());
  if (e == hipSuccess) e = up(L.eblocks, b->eblocks.data(), sizeof(HChunk) * b->eblocks.size());
  if (e == hipSuccess) e = up(L.crystal_order, b->crystal_order.data(), 4 * b->crystal_order.size());
  if (e == hipSuccess) e = up(L.sort_items, b->sort_items.data(), 4 * b->sort_items.size());
  if (e == hipSuccess) e = up(L.big_chunks, b->big_chunks.data(), sizeof(BigChunk) * b->big_chunks.size());
  if (e == hipSuccess) e = up(L.big_crystals, b->big_crystals.data(), sizeof(BigChunk) * b->big_crystals.size());
  if (e == hipSuccess) e = up(L.bw_items, b->bw_items.data(), sizeof(BwItem) * b->bw_items.size());
  if (e == hipSuccess) e = up(L.ab_items, b->ab_items.data(), sizeof(AbItem) * b->ab_items.size());
  if (e == hipSuccess) e = up(L.fam_ops, b->fam_ops.data(), sizeof(FamOps) * b->fam_ops.size());
  if (e == hipSuccess && b->rec) {
    e = up(L.sf_items_rec, b->sf_items_rec.data(), sizeof(SfItem) * b->sf_items_rec.size());
    if (e == hipSuccess) e = up(L.rec_of, b->use_rec.data(), 4 * b->use_rec.size());
  }
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("upload: ") + hipGetErrorString(e));
  launch_fill_i32(at<int32_t>(ws, L.err_flag), 1, 0, s);
  // pageable copies complete before return, but the tables stay owned by the
  // handle anyway; wait so that the handle may be destroyed right after
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("upload sync: ") + hipGetErrorString(e));
  b->last_ws = ws;
  return hip_check("upload");
}


int xrd_enumerate_hkl(xrd_batch *b, void *ws, const xrd_refl *r) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  const WsLayout &L = b->ws;
  b->sorted_ws = nullptr;
  b->sorted_tt = nullptr;
  b->deriv_ws = nullptr;
  b->deriv_h = nullptr;
  launch_enumerate(at<CrystalPlan>(ws, L.plan), b->desc.n_crystals, at<EnumChunk>(ws, L.enum_chunk_tab),
                   (int64_t)b->enum_chunks.size(), b->desc.wavelength, at<int32_t>(ws, L.enum_count),
                   at<int64_t>(ws, L.enum_prefix), at<int64_t>(ws, L.scan_part), r->h, r->k, r->l, r->q,
                   r->two_theta, r->lp, r->refl_offset, b->desc.n_species, b->desc.frac, b->desc.species,
                   b->desc.occ, b->desc.bfac, b->desc.sf_coeff, at<CoeffF>(ws, L.coeff_f),
                   at<AtomRec>(ws, L.atoms), at<AtomRot>(ws, L.rot), at<int32_t>(ws, L.atom_orig),
                   at<SpeciesRun>(ws, L.runs), at<int32_t>(ws, L.run_count), at<int32_t>(ws, L.err_flag),
                   b->max_enum_chunks, b->max_atoms, stream_of(b));
  b->last_ws = ws;
  return hip_check("enumerate");
}


// Arguments of the row-recurrence launch for items ``items`` (device) of
// which the first n_heavy take a block each.
static SfRecArgs rec_args(const xrd_batch *b, void *ws, const xrd_refl *r, const SfItem *items, int64_t n_items,
                          int64_t n_heavy) {
  const WsLayout &L = b->ws;
  SfRecArgs a;
  a.n_c = b->desc.n_crystals;
  a.items = items;
  a.n_items = n_items;
  a.n_heavy = n_heavy;
  a.eblocks = at<HChunk>(ws, L.eblocks);
  a.n_eblocks = (int64_t)b->eblocks.size();
  a.entry_cap = b->desc.friedel ? b->half_cap : b->refl_cap;
  a.plan = at<CrystalPlan>(ws, L.plan);
  a.refl_offset = r->refl_offset;
  a.h = r->h;
  a.k = r->k;
  a.l = r->l;
  a.q = r->q;
  a.lp = r->lp;
  a.atoms = at<AtomRec>(ws, L.atoms);
  a.rot = at<AtomRot>(ws, L.rot);
  a.runs = at<SpeciesRun>(ws, L.runs);
  a.run_count = at<int32_t>(ws, L.run_count);
  a.coeff = b->desc.sf_coeff;
  a.coeff_f = at<CoeffF>(ws, L.coeff_f);
  a.seg_cnt = at<int32_t>(ws, L.seg_cnt);
  a.seg_index = at<int64_t>(ws, L.seg_index);
  a.seg_part = at<int64_t>(ws, L.seg_part);
  a.seg_start = at<int32_t>(ws, L.seg_start);
  a.n_entries = at<int64_t>(ws, L.n_entries);
  a.rec_of = at<int32_t>(ws, L.rec_of);
  return a;
}

static Fork side_of(xrd_batch *b);

// The forward sums of the batch's current tables: the recurrence for its
// crystals (on the caller's stream) and the direct sum for the others (on a
// side stream when both run, joined before the call returns).
static void launch_forward_sums(xrd_batch *b, void *ws, const xrd_refl *r, void *A, void *B, double *I,
                                void *deriv) {
  const WsLayout &L = b->ws;
  hipStream_t s = stream_of(b);
  const bool mixed = b->desc.precision == XRD_MIXED, friedel = b->desc.friedel != 0;
  const int64_t nc = b->desc.n_crystals;
  const bool any_rec = b->n_rec > 0, any_direct = b->n_rec < nc;
  Fork f{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (any_rec && any_direct) f = side_of(b);
  hipStream_t sd = f.side ? f.side : s;
  if (f.side) {
    (void)hipEventRecord(f.fork, s);
    (void)hipStreamWaitEvent(f.side, f.fork, 0);
  }
  if (any_rec)
    launch_sf_rec(mixed, friedel,
                  rec_args(b, ws, r, at<SfItem>(ws, L.sf_items_rec), (int64_t)b->sf_items_rec.size(), b->sf_heavy_rec),
                  A, B, I, deriv, s);
  if (any_direct)
    launch_sf(mixed, friedel, at<SfItem>(ws, L.sf_items), (int64_t)b->sf_items.size(), b->sf_heavy,
              at<CrystalPlan>(ws, L.plan), r->refl_offset, r->h, r->k, r->l, r->q, r->lp, at<AtomRec>(ws, L.atoms),
              at<SpeciesRun>(ws, L.runs), at<int32_t>(ws, L.run_count), b->desc.sf_coeff, at<CoeffF>(ws, L.coeff_f),
              A, B, I, deriv, b->rpt, sd);
  if (f.side) {
    (void)hipEventRecord(f.join, f.side);
    (void)hipStreamWaitEvent(s, f.join, 0);
  }
}

int xrd_structure_factors(xrd_batch *b, void *ws, const xrd_refl *r, void *A, void *B, double *I) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (!A || !B || !I) return fail(XRD_ERR_INVALID_ARG, "A, B and I must be non-NULL");
  const WsLayout &L = b->ws;
  void *deriv = L.sf_deriv >= 0 ? at<char>(ws, L.sf_deriv) : nullptr;
  launch_forward_sums(b, ws, r, A, B, I, deriv);
  b->deriv_ws = deriv ? ws : nullptr;
  b->deriv_h = deriv ? r->h : nullptr;
  b->last_ws = ws;
  return hip_check("structure_factors");
}

static SortArgs sort_args(xrd_batch *b, void *ws, const WsLayout &L, const xrd_refl *r);

static void release_side(xrd_batch *b) {
  // teardown: a failure here leaves nothing to recover, so it is dropped
  for (hipEvent_t e : {b->ev_fork, b->ev_join, b->ev_join2})
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t st : {b->side, b->side2})
    if (st) (void)hipStreamDestroy(st);
  b->side = b->side2 = nullptr;
  b->ev_fork = b->ev_join = b->ev_join2 = nullptr;
  b->side_device = -1;
}

// The batch's side streams on the current device (default priority,
// non-blocking), or none if they cannot be made (then everything runs on the
// caller's stream).  They are made at the first call outside stream capture
// (making a stream would end a capture); a call captured before that runs on
// the caller's stream alone.
static Fork side_of(xrd_batch *b) {
  const Fork none{nullptr, nullptr, nullptr, nullptr, nullptr};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return none;
  if (b->side_device != dev) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream_of(b), &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      (void)hipGetLastError();
      return none;
    }
    release_side(b);
    bool ok = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&b->side2, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev_join2, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      release_side(b);
      (void)hipGetLastError();
      return none;
    }
    b->side_device = dev;
  }
  return Fork{b->side, b->side2, b->ev_fork, b->ev_join, b->ev_join2};
}

static void ensure_sorted(xrd_batch *b, void *ws, const xrd_refl *r) {
  if (b->sorted_ws == ws && b->sorted_tt == r->two_theta) return;
  launch_sort(sort_args(b, ws, b->ws, r), stream_of(b));
  b->sorted_ws = ws;
  b->sorted_tt = r->two_theta;
}

static SortArgs sort_args(xrd_batch *b, void *ws, const WsLayout &L, const xrd_refl *r) {
  SortArgs a;
  a.n_c = b->desc.n_crystals;
  a.plan = at<CrystalPlan>(ws, L.plan);
  a.refl_offset = r->refl_offset;
  a.tt = r->two_theta;
  a.h = r->h;
  a.k = r->k;
  a.l = r->l;
  a.bin_count = at<int32_t>(ws, L.bin_count);
  a.bin_start = at<int64_t>(ws, L.bin_start);
  a.n_bins = b->n_bins;
  a.skey = at<double>(ws, L.skey);
  a.sidx = at<int32_t>(ws, L.sidx);
  a.order = at<int32_t>(ws, L.crystal_order);
  a.n_small = b->n_small;
  a.items = at<int32_t>(ws, L.sort_items);
  a.friedel = b->desc.friedel != 0 ? 1 : 0;
  a.ent_key = at<double>(ws, L.ent_key);
  a.ent_idx = at<int32_t>(ws, L.ent_idx);
  a.big_chunks = at<BigChunk>(ws, L.big_chunks);
  a.n_big_chunks = (int64_t)b->big_chunks.size();
  a.big_crystals = at<BigChunk>(ws, L.big_crystals);
  a.n_big = (int64_t)b->big_crystals.size();
  a.big_cnt = at<int32_t>(ws, L.big_cnt);
  a.big_off = at<int64_t>(ws, L.big_off);
  a.big_np = at<int32_t>(ws, L.big_np);
  a.big_nb_max = b->big_nb_max;
  a.big_hist = at<int32_t>(ws, L.big_hist);
  a.big_boff = at<int64_t>(ws, L.big_boff);
  a.big_buckets = b->big_buckets;
  a.big_over = at<int2>(ws, L.big_over);
  return a;
}

static int check_merge_args(const xrd_refl *r, const double *I, const xrd_peaks *p) {
  if (int e = check_refl(r)) return e;
  if (!I || !p || !p->two_theta || !p->intensity || !p->scaled || !p->mult || !p->first || !p->perm ||
      !p->peak_offset)
    return fail(XRD_ERR_INVALID_ARG, "peak arrays and I must be non-NULL");
  return XRD_OK;
}

// Arguments of the merge kernels with the batch's tables and scratch at
// layout L in ``ws``.
static MergeArgs merge_args(xrd_batch *b, void *ws, const WsLayout &L, const xrd_refl *r, const double *I,
                            xrd_peaks *p) {
  MergeArgs a;
  a.sort = sort_args(b, ws, L, r);
  a.n_c = b->desc.n_crystals;
  a.tol = b->desc.merge_tol;
  a.thr = b->desc.rel_threshold;
  a.inten = I;
  a.flags = at<int32_t>(ws, L.flags);
  a.tmp_tt = at<double>(ws, L.tmp_tt);
  a.tmp_i = at<double>(ws, L.tmp_i);
  a.tmp_mult = at<int32_t>(ws, L.tmp_mult);
  a.tmp_first = at<int64_t>(ws, L.tmp_first);
  a.pk_count = at<int32_t>(ws, L.pk_count);
  a.peak_chunks = at<HChunk>(ws, L.peak_chunks);
  a.n_peak_chunks = (int64_t)b->peak_chunks.size();
  a.cmax = at<uint64_t>(ws, L.cmax);
  a.pk_tt = p->two_theta;
  a.pk_i = p->intensity;
  a.pk_y = p->scaled;
  a.pk_mult = p->mult;
  a.pk_first = p->first;
  a.perm = p->perm;
  a.peak_offset = p->peak_offset;
  return a;
}

int xrd_merge_peaks(xrd_batch *b, void *ws, const xrd_refl *r, const double *I, xrd_peaks *p) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_merge_args(r, I, p)) return e;
  // the merge sorts as it goes, and leaves the sorted order behind
  launch_merge(merge_args(b, ws, b->ws, r, I, p), stream_of(b));
  b->sorted_ws = ws;
  b->sorted_tt = r->two_theta;
  b->last_ws = ws;
  return hip_check("merge_peaks");
}

int xrd_merge_peaks_noalloc(xrd_batch *b, const xrd_refl *r, const double *I, xrd_peaks *p) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_merge_args(r, I, p)) return e;
  const WsLayout &M = b->mws;
  if (M.total > kNoallocBytes)
    return fail(XRD_ERR_CAPACITY, "the merge of this batch needs " + std::to_string(M.total) +
                                      " bytes of scratch; the fixed scratch holds " + std::to_string(kNoallocBytes));
  void *sp = nullptr;
  hipError_t e = noalloc_scratch(&sp);
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  // the batch's merge tables into this device's scratch (another call may have
  // left other contents there), then the merge on the caller's stream only
  hipStream_t s = stream_of(b);
  auto up = [&](int64_t off, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(at<char>(sp, off), src, bytes, hipMemcpyHostToDevice, s);
  };
  e = up(M.plan, b->plan.data(), sizeof(CrystalPlan) * b->plan.size());
  if (e == hipSuccess) e = up(M.peak_chunks, b->peak_chunks.data(), sizeof(HChunk) * b->peak_chunks.size());
  if (e == hipSuccess) e = up(M.crystal_order, b->crystal_order.data(), 4 * b->crystal_order.size());
  if (e == hipSuccess) e = up(M.sort_items, b->sort_items.data(), 4 * b->sort_items.size());
  if (e == hipSuccess) e = up(M.big_chunks, b->big_chunks.data(), sizeof(BigChunk) * b->big_chunks.size());
  if (e == hipSuccess) e = up(M.big_crystals, b->big_crystals.data(), sizeof(BigChunk) * b->big_crystals.size());
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("scratch tables: ") + hipGetErrorString(e));
  launch_merge(merge_args(b, sp, M, r, I, p), s);
  // the sorted order went to the scratch, which later calls may overwrite
  b->sorted_ws = nullptr;
  b->sorted_tt = nullptr;
  return hip_check("merge_peaks_noalloc");
}

static int check_grid(const xrd_grid *g) {
  if (!g) return fail(XRD_ERR_INVALID_ARG, "grid is NULL");
  if (!(g->n_points >= 1) || !(g->dt > 0.0) || !(g->sigma > 0.0) || !(g->window_sigmas > 0.0) ||
      !std::isfinite(g->t0) || !std::isfinite(g->dt) || !std::isfinite(g->sigma) || !std::isfinite(g->window_sigmas))
    return fail(XRD_ERR_INVALID_ARG, "grid needs n_points >= 1, dt > 0, sigma > 0, window_sigmas > 0");
  if (g->n_points >= ((int64_t)1 << 31) || g->dt < 1e-9 || std::fabs(g->t0) > 1e6 || g->window_sigmas > 30.0 ||
      g->window_sigmas * g->sigma > 1e3)
    return fail(XRD_ERR_INVALID_ARG, "grid out of range: n_points <= 2^31, dt >= 1e-9, |t0| <= 1e6, "
                                     "window_sigmas <= 30, window <= 1000 deg");
  return XRD_OK;
}

int xrd_pattern_forward(xrd_batch *b, void *ws, const xrd_refl *r, const double *I, const xrd_grid *g, double *y) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (int e = check_grid(g)) return e;
  if (!I || !y) return fail(XRD_ERR_INVALID_ARG, "I and y must be non-NULL");
  if (g->n_points > b->grid_cap)
    return fail(XRD_ERR_INVALID_ARG, "n_points exceeds the batch's grid_capacity (" + std::to_string(b->grid_cap) + ")");
  ensure_sorted(b, ws, r);
  const WsLayout &L = b->ws;
  launch_broaden_fwd(b->desc.precision == XRD_MIXED, at<HChunk>(ws, L.eblocks),
                     (int64_t)b->eblocks.size(), at<CrystalPlan>(ws, L.plan),
                     at<int32_t>(ws, L.crystal_order), b->desc.n_crystals,
                     b->desc.friedel != 0, r->refl_offset, at<double>(ws, L.ent_key), at<int32_t>(ws, L.ent_idx), I,
                     g->t0, g->dt, g->n_points, g->sigma, g->window_sigmas, b->span_cap, at<double>(ws, L.ent_w),
                     at<int32_t>(ws, L.span_first), at<int32_t>(ws, L.span_last), y, stream_of(b));
  b->last_ws = ws;
  return hip_check("pattern_forward");
}

int xrd_pattern_backward(xrd_batch *b, void *ws, const xrd_refl *r, const xrd_grid *g, const double *dL_dy,
                         double *dL_dfrac, double *dL_dbfac, double *dL_dlattice) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (int e = check_grid(g)) return e;
  if (!dL_dy || !dL_dlattice || (b->n_atoms > 0 && (!dL_dfrac || !dL_dbfac)))
    return fail(XRD_ERR_INVALID_ARG, "gradient buffers must be non-NULL");
  if (b->desc.forward_only) return fail(XRD_ERR_UNSUPPORTED, "the batch was created forward_only (no adjoint tables)");
  const WsLayout &L = b->ws;
  hipStream_t s = stream_of(b);
  const bool mixed = b->desc.precision == XRD_MIXED, friedel = b->desc.friedel != 0;
  const CrystalPlan *plan = at<CrystalPlan>(ws, L.plan);
  const SfItem *items = at<SfItem>(ws, L.sf_items_bw);
  const int64_t n_items = (int64_t)b->sf_items_bw.size();
  double2 *w12 = at<double2>(ws, L.bw_w12);
  double *ga = at<double>(ws, L.bw_ga), *gb = at<double>(ws, L.bw_gb), *dq = at<double>(ws, L.bw_dq);
  ensure_sorted(b, ws, r);
  const void *deriv = (L.sf_deriv >= 0 && b->deriv_ws == ws && b->deriv_h == r->h) ? at<char>(ws, L.sf_deriv) : nullptr;
  launch_broaden_adj(mixed, at<HChunk>(ws, L.eblocks), (int64_t)b->eblocks.size(), plan, friedel,
                     r->refl_offset, at<double>(ws, L.ent_key), at<int32_t>(ws, L.ent_idx), dL_dy, g->t0, g->dt,
                     g->n_points, g->sigma, g->window_sigmas, w12, s);
  launch_sf_bw(mixed, friedel, items, n_items, b->sf_heavy_bw, plan, r->refl_offset, r->h, r->k, r->l, r->q, r->lp,
               b->desc.wavelength, at<AtomRec>(ws, L.atoms), at<SpeciesRun>(ws, L.runs), at<int32_t>(ws, L.run_count),
               b->desc.sf_coeff, at<CoeffF>(ws, L.coeff_f), deriv, w12, ga, gb, dq, at<double>(ws, L.bw_part6),
               at<double>(ws, L.bw_partf), b->rpt, s);
  launch_atom_bw(mixed, friedel, at<BwItem>(ws, L.bw_items), (int64_t)b->bw_items.size(), plan, r->refl_offset,
                 r->h, r->k, r->l, r->q, ga, gb, at<AtomRec>(ws, L.atoms), at<SpeciesRun>(ws, L.runs),
                 at<int32_t>(ws, L.run_count), b->desc.sf_coeff, at<CoeffF>(ws, L.coeff_f), b->bw_tile, b->runs_cap_max,
                 at<double>(ws, L.bw_part), s);
  launch_bw_finish(at<AbItem>(ws, L.ab_items), (int64_t)b->ab_items.size(), friedel, plan, b->desc.n_crystals,
                   r->refl_offset, at<double>(ws, L.bw_part), at<double>(ws, L.bw_partf), at<int32_t>(ws, L.atom_orig),
                   at<double>(ws, L.bw_part6), dL_dfrac, dL_dbfac, dL_dlattice, s);
  b->last_ws = ws;
  return hip_check("pattern_backward");
}

int xrd_autotune(xrd_batch *b, void *ws, const xrd_refl *r, int32_t *split_out) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  const WsLayout &L = b->ws;
  hipStream_t s = stream_of(b);
  const bool mixed = b->desc.precision == XRD_MIXED, friedel = b->desc.friedel != 0;
  const CrystalPlan *plan = at<CrystalPlan>(ws, L.plan);
  // outputs of the timing runs: A, B and I go to the merge's staging scratch
  // (each merge rewrites it before reading it), derivatives (when kept) to
  // their usual place
  void *A = at<void>(ws, L.tmp_tt), *B = at<void>(ws, L.tmp_i);
  double *I = at<double>(ws, L.tmp_first);
  void *deriv = L.sf_deriv >= 0 ? at<char>(ws, L.sf_deriv) : nullptr;
  const bool adjoint = !b->desc.forward_only;
  double2 *w12 = adjoint ? at<double2>(ws, L.bw_w12) : nullptr;
  const int64_t nc = b->desc.n_crystals;
  auto run_bw = [&](const std::vector<SfItem> &t, int64_t nh) {
    launch_sf_bw(mixed, friedel, at<SfItem>(ws, L.sf_items_bw), (int64_t)t.size(), nh, plan, r->refl_offset, r->h,
                 r->k, r->l, r->q, r->lp, b->desc.wavelength, at<AtomRec>(ws, L.atoms), at<SpeciesRun>(ws, L.runs),
                 at<int32_t>(ws, L.run_count), b->desc.sf_coeff, at<CoeffF>(ws, L.coeff_f), deriv, w12,
                 at<double>(ws, L.bw_ga), at<double>(ws, L.bw_gb), at<double>(ws, L.bw_dq), at<double>(ws, L.bw_part6),
                 at<double>(ws, L.bw_partf), b->rpt, s);
  };
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  // median of five launches after one untimed launch
  auto timed = [&](auto &&launch) -> float {
    float t[5] = {0, 0, 0, 0, 0};
    launch();
    for (int i = 0; i < 5 && e == hipSuccess; ++i) {
      e = hipEventRecord(ev[0], s);
      launch();
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&t[i], ev[0], ev[1]);
    }
    std::sort(t, t + 5);
    return t[2];
  };
  // the forward tables (both methods) and the per-crystal choice into the workspace
  auto upload_fwd = [&]() {
    if (e == hipSuccess && !b->sf_items.empty())
      e = hipMemcpyAsync(at<char>(ws, L.sf_items), b->sf_items.data(), sizeof(SfItem) * b->sf_items.size(),
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess && b->rec && !b->sf_items_rec.empty())
      e = hipMemcpyAsync(at<char>(ws, L.sf_items_rec), b->sf_items_rec.data(),
                         sizeof(SfItem) * b->sf_items_rec.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && b->rec)
      e = hipMemcpyAsync(at<char>(ws, L.rec_of), b->use_rec.data(), 4 * b->use_rec.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  };
  auto time_fwd = [&]() -> float {
    upload_fwd();
    if (e != hipSuccess) return 0.f;
    const float ms = timed([&] { launch_forward_sums(b, ws, r, A, B, I, deriv); });
    if (e == hipSuccess) e = hipGetLastError();
    return ms;
  };
  // candidate thresholds; those giving the same tables as an earlier one are skipped
  const int32_t cand[] = {8, 16, 24, 32, 48, 64, 96, 128, 256, 512, INT32_MAX};
  // At the current tile shape: the recurrence threshold (XRD_SF_AUTO) and the
  // forward split, then the adjoint's split; leaves the best of each in the
  // batch and returns the sum of the two times (the forward's alone without
  // an adjoint).
  auto tune_shape = [&]() -> float {
    float fwd_best = 0.f, bw_best = 0.f;
    // (XRD_SF_AUTO) which crystals take the recurrence: atom thresholds
    if (b->desc.sf_method == XRD_SF_AUTO) {
      const int32_t rcand[] = {64, 128, 256, 512, 1024, INT32_MAX};
      std::vector<int64_t> seen;
      float best = 0.f;
      int32_t best_t = b->rec_min_atoms;
      for (int32_t t : rcand) {
        if (e != hipSuccess) break;
        b->rec_min_atoms = t;
        choose_methods(b);
        if (std::find(seen.begin(), seen.end(), b->n_rec) != seen.end()) continue;
        seen.push_back(b->n_rec);
        const float ms = time_fwd();
        if (e == hipSuccess && (seen.size() == 1 || ms < best)) {
          best = ms;
          best_t = t;
        }
      }
      b->rec_min_atoms = best_t;
      choose_methods(b);
    }
    // split-K of the forward sums
    {
      std::vector<std::pair<int64_t, int64_t>> seen;
      int32_t best_split = b->split_fwd;
      for (int32_t c : cand) {
        if (e != hipSuccess) break;
        b->split_fwd = c;
        choose_methods(b);
        const std::pair<int64_t, int64_t> key{b->sf_heavy, b->sf_heavy_rec};
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
        seen.push_back(key);
        const float ms = time_fwd();
        if (e == hipSuccess && (seen.size() == 1 || ms < fwd_best)) {
          fwd_best = ms;
          best_split = c;
        }
      }
      b->split_fwd = best_split;
      choose_methods(b);
      upload_fwd();
    }
    if (!adjoint) return fwd_best;
    // the adjoint's inputs: derivatives of the chosen forward tables, zero grid weights
    if (e == hipSuccess) {
      launch_forward_sums(b, ws, r, A, B, I, deriv);
      launch_fill_u64(reinterpret_cast<uint64_t *>(w12), 2 * b->refl_cap, 0, s);
      e = hipGetLastError();
    }
    std::vector<SfItem> t;
    std::vector<int64_t> seen;
    for (int32_t c : cand) {
      if (e != hipSuccess) break;
      const int64_t nh = sf_table(b, c, &t);
      if (std::find(seen.begin(), seen.end(), nh) != seen.end()) continue;
      seen.push_back(nh);
      e = hipMemcpyAsync(at<char>(ws, L.sf_items_bw), t.data(), sizeof(SfItem) * t.size(), hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) break;
      const float ms = timed([&] { run_bw(t, nh); });
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess && (seen.size() == 1 || ms < bw_best)) {
        bw_best = ms;
        b->split_bw = c;
      }
    }
    return fwd_best + bw_best;
  };
  // the tile shape (reflections per lane), unless the batch fixed it: each
  // shape with its own best splits, the fastest forward plus adjoint kept
  auto upload_plan = [&]() {
    if (e == hipSuccess)
      e = hipMemcpyAsync(at<char>(ws, L.plan), b->plan.data(), sizeof(CrystalPlan) * b->plan.size(),
                         hipMemcpyHostToDevice, s);
  };
  if (nc > 0 && e == hipSuccess) {
    std::vector<int32_t> shapes = {1, 2, 4};
    if (b->desc.sf_rpt != 0) shapes = {b->desc.sf_rpt};
    struct Choice {
      int32_t rpt, split_fwd, split_bw, rec_min_atoms;
    } best{b->rpt, b->split_fwd, b->split_bw, b->rec_min_atoms};
    float best_ms = 0.f;
    bool first = true;
    for (int32_t rpt : shapes) {
      if (e != hipSuccess) break;
      set_tiles(b, rpt);
      upload_plan();
      const float ms = tune_shape();
      if (e == hipSuccess && (first || ms < best_ms)) {
        best_ms = ms;
        best = Choice{rpt, b->split_fwd, b->split_bw, b->rec_min_atoms};
        first = false;
      }
    }
    set_tiles(b, best.rpt);
    b->split_fwd = best.split_fwd;
    b->split_bw = best.split_bw;
    b->rec_min_atoms = best.rec_min_atoms;
    choose_methods(b);
    upload_plan();
    upload_fwd();
    if (adjoint) {
      b->sf_heavy_bw = sf_table(b, b->split_bw, &b->sf_items_bw);
      if (e == hipSuccess)
        e = hipMemcpyAsync(at<char>(ws, L.sf_items_bw), b->sf_items_bw.data(), sizeof(SfItem) * b->sf_items_bw.size(),
                           hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  // the timing runs overwrote the kept derivatives' record of the last call
  b->deriv_ws = nullptr;
  b->deriv_h = nullptr;
  b->last_ws = ws;
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
  if (split_out) {
    split_out[0] = b->split_fwd;
    split_out[1] = b->split_bw;
    if (b->desc.sf_method == XRD_SF_AUTO) split_out[2] = b->rec_min_atoms;
  }
  return XRD_OK;
}

int xrd_batch_get_sf_rpt(const xrd_batch *b, int32_t *rpt) {
  if (!b || !rpt) return fail(XRD_ERR_INVALID_ARG, "batch or rpt is NULL");
  *rpt = b->rpt;
  return XRD_OK;
}

int xrd_preferred_orientation(xrd_batch *b, void *ws, const xrd_refl *r, const double *hp, const double *march_r,
                              double *I) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (!I || (b->desc.n_crystals > 0 && (!hp || !march_r)))
    return fail(XRD_ERR_INVALID_ARG, "hp, march_r and I must be non-NULL");
  const WsLayout &L = b->ws;
  launch_march_dollase(at<HChunk>(ws, L.peak_chunks), (int64_t)b->peak_chunks.size(), at<CrystalPlan>(ws, L.plan),
                       r->refl_offset, r->h, r->k, r->l, hp, march_r, I, stream_of(b));
  b->last_ws = ws;
  return hip_check("preferred_orientation");
}

int xrd_peak_families(xrd_batch *b, void *ws, const xrd_refl *r, const xrd_peaks *p, int32_t rule,
                      int32_t *n_families, int32_t *family_of, int64_t *family_label, int32_t *family_mult) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (!p || !p->mult || !p->first || !p->perm || !p->peak_offset)
    return fail(XRD_ERR_INVALID_ARG, "peak arrays must be non-NULL");
  if (rule != XRD_FAMILY_INDICES && rule != XRD_FAMILY_LATTICE) return fail(XRD_ERR_INVALID_ARG, "unknown rule");
  if (!n_families || !family_of || !family_label || !family_mult)
    return fail(XRD_ERR_INVALID_ARG, "family arrays must be non-NULL");
  launch_peak_families(at<HChunk>(ws, b->ws.peak_chunks), (int64_t)b->peak_chunks.size(), at<FamOps>(ws, b->ws.fam_ops),
                       p->peak_offset, p->first,
                       p->mult, p->perm, r->h, r->k, r->l, rule, n_families, family_of, family_label, family_mult,
                       stream_of(b));
  b->last_ws = ws;
  return hip_check("peak_families");
}

int xrd_combine_lines(int64_t n_crystals, const xrd_line *line0, const xrd_line *line1, xrd_line_peaks *out,
                      void *stream) {
  if (n_crystals < 0) return fail(XRD_ERR_INVALID_ARG, "n_crystals < 0");
  if (!line0 || !out) return fail(XRD_ERR_INVALID_ARG, "line0 and out must be non-NULL");
  auto check_line = [](const xrd_line *l) -> int {
    const xrd_peaks *p = l->peaks;
    if (!p || !l->q || !p->two_theta || !p->intensity || !p->mult || !p->first || !p->perm || !p->peak_offset)
      return fail(XRD_ERR_INVALID_ARG, "a line's peak arrays and q must be non-NULL");
    if (!std::isfinite(l->weight) || l->weight < 0.0) return fail(XRD_ERR_INVALID_ARG, "line weights must be >= 0");
    return XRD_OK;
  };
  if (int e = check_line(line0)) return e;
  if (line1)
    if (int e = check_line(line1)) return e;
  if (!out->two_theta || !out->intensity || !out->scaled || !out->mult || !out->d || !out->line || !out->source ||
      !out->peak_offset)
    return fail(XRD_ERR_INVALID_ARG, "output arrays must be non-NULL");
  auto lp = [](const xrd_line *l) {
    const xrd_peaks *p = l->peaks;
    return LinePeaks{p->two_theta, p->intensity, l->q, p->mult, p->first, p->perm, p->peak_offset, l->weight};
  };
  const LinePeaks p0 = lp(line0);
  LinePeaks p1{};
  if (line1) p1 = lp(line1);
  const LineOut o{out->two_theta, out->intensity, out->scaled, out->mult,
                  out->d,         out->line,      out->source, out->peak_offset};
  launch_combine_lines(n_crystals, p0, line1 ? &p1 : nullptr, o, reinterpret_cast<hipStream_t>(stream));
  return hip_check("combine_lines");
}

int xrd_pattern_caglioti(xrd_batch *b, void *ws, const xrd_refl *r, const double *I, const xrd_grid *g, double U,
                         double V, double W, double eta, double *y) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (int e = check_ws(b, ws)) return e;
  if (int e = check_refl(r)) return e;
  if (int e = check_grid(g)) return e;
  if (!I || !y) return fail(XRD_ERR_INVALID_ARG, "I and y must be non-NULL");
  if (!std::isfinite(U) || !std::isfinite(V) || !std::isfinite(W))
    return fail(XRD_ERR_INVALID_ARG, "U, V and W must be finite");
  if (!(eta >= 0.0 && eta <= 1.0)) return fail(XRD_ERR_INVALID_ARG, "eta must lie in [0, 1]");
  ensure_sorted(b, ws, r);
  const WsLayout &L = b->ws;
  launch_broaden_caglioti(b->desc.precision == XRD_MIXED, at<CrystalPlan>(ws, L.plan), b->desc.n_crystals, r->refl_offset, b->desc.friedel != 0,
                          at<double>(ws, L.ent_key), at<int32_t>(ws, L.ent_idx), I, g->t0, g->dt, g->n_points, U, V,
                          W, eta, g->window_sigmas, y, stream_of(b));
  b->last_ws = ws;
  return hip_check("pattern_caglioti");
}

int xrd_pattern_noise(xrd_batch *b, int64_t n_points, uint64_t seed, double rel, double abs, double *y) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  if (!y) return fail(XRD_ERR_INVALID_ARG, "y is NULL");
  if (n_points < 1 || n_points > b->grid_cap)
    return fail(XRD_ERR_INVALID_ARG, "n_points must be in [1, grid_capacity]");
  if (!(rel >= 0.0) || !(abs >= 0.0) || !std::isfinite(rel) || !std::isfinite(abs))
    return fail(XRD_ERR_INVALID_ARG, "rel and abs must be finite and >= 0");
  launch_noise(b->desc.n_crystals * n_points, seed, rel, abs, y, stream_of(b));
  return hip_check("pattern_noise");
}

int xrd_read_counts(xrd_batch *b, const xrd_refl *r, const xrd_peaks *p, int64_t *host_refl_offset,
                    int64_t *host_peak_offset) {
  if (!b) return fail(XRD_ERR_INVALID_ARG, "batch is NULL");
  hipStream_t s = stream_of(b);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
  const size_t n = (size_t)(b->desc.n_crystals + 1) * sizeof(int64_t);
  if (host_refl_offset) {
    if (!r || !r->refl_offset) return fail(XRD_ERR_INVALID_ARG, "refl_offset is NULL");
    e = hipMemcpy(host_refl_offset, r->refl_offset, n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("copy refl_offset: ") + hipGetErrorString(e));
  }
  if (host_peak_offset) {
    if (!p || !p->peak_offset) return fail(XRD_ERR_INVALID_ARG, "peak_offset is NULL");
    e = hipMemcpy(host_peak_offset, p->peak_offset, n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("copy peak_offset: ") + hipGetErrorString(e));
  }
  if (b->last_ws) {
    int32_t flag = 0;
    e = hipMemcpy(&flag, at<int32_t>(b->last_ws, b->ws.err_flag), 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(XRD_ERR_HIP, std::string("copy error flag: ") + hipGetErrorString(e));
    if (flag) return fail(XRD_ERR_INVALID_ARG, "a species index was outside [0, n_species)");
  }
  return XRD_OK;
}

void xrd_batch_destroy(xrd_batch *b) {
  if (!b) return;
  release_side(b);
  delete b;
}

}  // extern "C"
