// Reciprocal-lattice enumeration inside the limiting sphere (paper, Section
// 2: generation of the reciprocal lattice points within the physically
// accessible sphere), with the per-reflection geometry q, 2theta and the
// Lorentz-polarisation factor.
//
// Each crystal's search box [-H,H]x[-K,K]x[-L,L] is split at the origin; only
// the points above it in lexicographic order are visited, since (h,k,l) and
// (-h,-k,-l) share q, 2theta and LP bit for bit.  The half box is taken row
// by row ((h, k) fixed, one row per thread), each row only over the l that
// the quadratic q(l) can bring into the limiting sphere.  The rows are taken
// in chunks of 64, one wavefront each: count the survivors per chunk, scan
// the counts, then flatten the chunk's rows into candidate points, test,
// rank and write each survivor (h, k, l, q, 2theta, LP) and its Friedel
// mate.  The output of a crystal is its full sphere shell in ascending
// (h, k, l) order:
// the positive half occupies the upper half of the segment and mate i sits at
// the mirror position, so no sort is needed for the hkl listing.
//
// q and 2theta are evaluated in double precision in a fixed order with FMA
// contraction off, as the definition writes them.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
static_assert(kEnumRows <= 64, "one row per lane of a wavefront");
constexpr double kPi = 3.14159265358979323846;
constexpr size_t kFusedPackLds = 4096;  // largest cursor space the fused count-and-pack launch carries
constexpr int64_t kFusedPackAtoms = 1024;  // largest crystal the fused launch packs (one batch of records in flight)

struct Hkl {
  int h, k, l;
};

__device__ __forceinline__ double q_of(const CrystalPlan &P, const Hkl &m) {
#pragma clang fp contract(off)
  const double h = m.h, k = m.k, l = m.l;
  const double hh = h * h, kk = k * k, ll = l * l, hk = h * k, hl = h * l, kl = k * l;
  return P.gs[0] * hh + P.gs[1] * kk + P.gs[2] * ll + 2.0 * (P.gs[3] * hk + P.gs[4] * hl + P.gs[5] * kl);
}

// 2theta (deg) of q; negative when sin(theta) would exceed 1.
__device__ __forceinline__ double two_theta_of(double q, double lambda) {
#pragma clang fp contract(off)
  const double s = 0.5 * lambda * sqrt(q);
  if (s > 1.0) return -1.0;
  return 2.0 * asin(s) * (180.0 / kPi);
}

// Row rho of a crystal's positive half: the half box above the origin in
// lexicographic (h, k, l) order is the row (0, 0) with l in [1, L], the rows
// (0, k) for k in [1, K], then (h, k) for h in [1, H], k in [-K, K], each with
// l in [-L, L] (h outermost).  Rows in this order, l ascending within a row,
// list the half in lexicographic order.
struct Row {
  int h, k, l0, l1;
};
__device__ __forceinline__ int64_t rows_of(const CrystalPlan &P) {
  return (int64_t)P.H * (2 * P.K + 1) + P.K + 1;
}
__device__ __forceinline__ Row row_of(const CrystalPlan &P, int64_t rho) {
  Row r;
  if (rho <= P.K) {
    r.h = 0;
    r.k = (int)rho;
  } else {
    const uint32_t nk = 2 * P.K + 1, x = (uint32_t)(rho - (P.K + 1)), hq = x / nk;
    r.h = 1 + (int)hq;
    r.k = (int)(x - hq * nk) - P.K;
  }
  r.l0 = (r.h == 0 && r.k == 0) ? 1 : -P.L;
  r.l1 = P.L;
  return r;
}

// The l of a row that can lie in the limiting sphere: q(l) = G33 l^2 +
// 2 (G13 h + G23 k) l + q(h, k, 0) is convex in l, so {q <= qhi} is an
// interval, bounded by the roots of the quadratic (qhi widened by 1e-9, and
// one more l on each side, so that rounding in the roots cannot drop a point;
// every candidate then takes the exact test).
__device__ __forceinline__ void row_candidates(const CrystalPlan &P, const Row &r, int *lo, int *hi) {
  const double h = r.h, k = r.k;
  const double A = P.gs[2];
  const double B = 2.0 * (P.gs[4] * h + P.gs[5] * k);
  const double C = P.gs[0] * h * h + P.gs[1] * k * k + 2.0 * P.gs[3] * h * k;
  const double disc = B * B - 4.0 * A * (C - P.qhi * (1.0 + 1e-9));
  if (!(disc >= 0.0)) {
    *lo = 1;
    *hi = 0;
    return;
  }
  const double sq = sqrt(disc), lim = (double)P.L + 1.0;
  const double r1 = fmin(fmax((-B - sq) / (2.0 * A), -lim), lim);
  const double r2 = fmin(fmax((-B + sq) / (2.0 * A), -lim), lim);
  *lo = max(r.l0, (int)floor(r1));
  *hi = min(r.l1, (int)ceil(r2));
}

// The test that defines a reflection: q in the prefilter band and 2theta in
// [tmin, tmax].  Inside the band narrowed by 3e-9 (relative) 2theta lies in
// range with a margin far above its rounding error, so 2theta is evaluated
// there only when wanted; the decision is the same either way, and the count
// and the fill take it with this one function.
__device__ __forceinline__ bool keep_point(const CrystalPlan &P, const Hkl &m, double lambda, bool want_tt, double *q,
                                           double *tt) {
  *q = q_of(P, m);
  if (*q < P.qlo || *q > P.qhi) return false;
  const bool inner = *q >= P.qlo * (1.0 + 3e-9) && *q <= P.qhi * (1.0 - 3e-9);
  if (inner && !want_tt) return true;
  *tt = two_theta_of(*q, lambda);
  return inner || (*tt >= P.tmin && *tt <= P.tmax);
}

// Survivors of one row.
__device__ __forceinline__ int row_count(const CrystalPlan &P, const Row &r, double lambda) {
  int lo, hi;
  row_candidates(P, r, &lo, &hi);
  int n = 0;
  for (int l = lo; l <= hi; ++l) {
    double q, tt;
    n += keep_point(P, Hkl{r.h, r.k, l}, lambda, false, &q, &tt) ? 1 : 0;
  }
  return n;
}

// LP = (1 + cos^2 2theta) / (sin^2 theta cos theta) from q directly:
// sin^2 theta = lambda^2 q / 4 (Bragg's law), cos 2theta = 1 - 2 sin^2 theta,
// cos theta = sqrt(1 - sin^2 theta); the same function of theta without the
// trigonometric round trip.
__device__ __forceinline__ double lp_of_q(double q, double lambda) {
#pragma clang fp contract(off)
  const double s2 = 0.25 * (lambda * lambda) * q;
  const double c2 = 1.0 - 2.0 * s2;
  return (1.0 + c2 * c2) / (s2 * sqrt(1.0 - s2));
}

// ---- atom packing ----------------------------------------------------------
//
// The structure-factor kernels read each crystal's atoms grouped by species
// (so that the scattering factor is evaluated once per species and
// reflection), as 48-byte records.  One wavefront packs one crystal: species
// histogram in LDS, ascending-species runs, then a stable scatter (an atom's
// slot is its species cursor plus the lanes of its species below it, the
// lanes of a species found by ballots over the species bits).  The wavefront works alone: it orders its
// LDS accesses with wavefront-scope fences, so several crystals can share a
// block.  The wavefront of crystal 0 also writes the single-precision
// coefficient table of the mixed path.

constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes of the wavefront holding the same species as this one (among the
// active lanes), by one ballot per bit that tells the species apart.
__device__ __forceinline__ uint64_t same_species(bool active, int sp, int nbits) {
  uint64_t m = __ballot(active);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (sp >> b) & 1;
    const uint64_t bal = __ballot(active && bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

struct AtomIn {
  int sp;
  double x, y, z, occ, bfac;
};

__device__ __forceinline__ AtomIn load_atom(int64_t j, int64_t a1, const double *__restrict__ frac,
                                            const int32_t *__restrict__ species, const double *__restrict__ occ,
                                            const double *__restrict__ bfac) {
  AtomIn r{-1, 0.0, 0.0, 0.0, 1.0, 0.0};
  if (j < a1) {
    r.sp = species[j];
    r.x = frac[3 * j];
    r.y = frac[3 * j + 1];
    r.z = frac[3 * j + 2];
    r.occ = occ[j];
    r.bfac = bfac[j];
  }
  return r;
}

// D: batches of 64 atom records in flight ahead of the one being placed
// (and 4 D batches of species per histogram round); larger D hides more of
// the loads' latency on crystals of many atoms at the cost of registers.
// NW: wavefronts of the block that pack the crystal together.  Wavefront w
// takes the w-th contiguous slice of its atoms (whole batches of 64) and
// counts their species into its own cursors (``cursor`` holds NW arrays of
// n_species); one exclusive scan over (species, wavefront) in that order
// then gives each wavefront its slots, so the atoms land where a single
// wavefront would place them.
template <int NW>
__device__ __forceinline__ void pack_sync() {
  if constexpr (NW > 1)
    __syncthreads();
  else
    wave_sync();
}

template <int D, int NW>
__device__ void pack_crystal(int c, int lane, int32_t *cursor, const CrystalPlan *__restrict__ plan,
                             int32_t n_species, const double *__restrict__ frac,
                             const int32_t *__restrict__ species, const double *__restrict__ occ,
                             const double *__restrict__ bfac, const double *__restrict__ coeff,
                             CoeffF *__restrict__ coeff_f, AtomRec *__restrict__ atoms,
                             AtomRot *__restrict__ rot, int32_t *__restrict__ orig, SpeciesRun *__restrict__ runs,
                             int32_t *__restrict__ run_count, int32_t *__restrict__ err) {
  const int w = NW > 1 ? (int)(threadIdx.x >> 6) : 0;
  if (c == 0 && w == 0) {
    // the single-precision coefficient table of the mixed path (one
    // rounding from double of each stored product)
    for (int t = lane; t < n_species; t += 64) {
      const double *c9 = coeff + 9 * t;
      CoeffF cf{};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cf.a[i] = (float)c9[i];
        cf.nbl[i] = (float)(-c9[4 + i] * 1.4426950408889634);
        cf.nab[i] = (float)(-c9[i] * c9[4 + i]);
      }
      cf.c = (float)c9[8];
      coeff_f[t] = cf;
    }
  }
  const CrystalPlan &P = plan[c];
  const int64_t a0 = P.atom_begin, a1 = P.atom_end;
  const int64_t per = ((a1 - a0 + NW - 1) / NW + 63) / 64 * 64;
  const int64_t s0 = min(a1, a0 + w * per), s1 = min(a1, s0 + per);  // this wavefront's atoms
  int32_t *const mine = cursor + w * n_species;
  const int nbits = n_species > 1 ? 32 - __builtin_clz((uint32_t)(n_species - 1)) : 0;
  for (int t = lane; t < n_species; t += 64) mine[t] = 0;
  wave_sync();
  // species histogram: the lowest lane of each species group adds its size
  for (int64_t base = s0; base < s1; base += 256 * D) {
    int sp[4 * D];
#pragma unroll
    for (int u = 0; u < 4 * D; ++u) {
      const int64_t j = base + 64 * u + lane;
      sp[u] = j < s1 ? species[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4 * D; ++u) {
      const bool active = base + 64 * u + lane < s1;
      if (active && (sp[u] < 0 || sp[u] >= n_species)) {
        atomicOr(err, 1);
        sp[u] = 0;
      }
      const uint64_t m = same_species(active, sp[u], nbits);
      if (active && lanes_below(m) == 0) mine[sp[u]] += __popcll(m);
      wave_sync();
    }
  }
  pack_sync<NW>();
  // ascending-species runs and each wavefront's cursors (exclusive scan
  // over species, then wavefronts), by wavefront 0
  if (w == 0) {
    int64_t running = a0;
    int nruns = 0;
    for (int t0 = 0; t0 < n_species; t0 += 64) {
      const int t = t0 + lane;
      int hw[NW], v = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        hw[q] = t < n_species ? cursor[q * n_species + t] : 0;
        v += hw[q];
      }
      int inc = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
      }
      const int tot = __shfl(inc, 63, 64);
      const uint64_t nz = __ballot(v > 0);
      const int rank = lanes_below(nz);
      const int64_t start = running + inc - v;
      if (v > 0) {
        SpeciesRun r;
        r.begin = (int32_t)start;
        r.end = (int32_t)(start + v);
        r.species = t;
        r.local = nruns + rank;
        runs[P.run_begin + nruns + rank] = r;
      }
      if (t < n_species) {
        int64_t o = start;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          cursor[q * n_species + t] = (int32_t)o;
          o += hw[q];
        }
      }
      wave_sync();
      running += tot;
      nruns += __popcll(nz);
    }
    if (lane == 0) run_count[c] = nruns;
  }
  pack_sync<NW>();
  // scatter in input order within each species: an atom's slot is its
  // species cursor plus the lanes of its species below it; the next D
  // batches of 64 atoms' records load while these are placed
  AtomIn cur[D];
#pragma unroll
  for (int u = 0; u < D; ++u) cur[u] = load_atom(s0 + 64 * u + lane, s1, frac, species, occ, bfac);
  for (int64_t batch = s0; batch < s1; batch += 64 * D) {
    AtomIn nxt[D];
#pragma unroll
    for (int u = 0; u < D; ++u) nxt[u] = load_atom(batch + 64 * (D + u) + lane, s1, frac, species, occ, bfac);
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int64_t base = batch + 64 * u;
      if (base >= s1) break;
      const AtomIn &in = cur[u];
      const int64_t j = base + lane;
      const bool active = j < s1;
      const int sp = active ? (in.sp < 0 || in.sp >= n_species ? 0 : in.sp) : 0;
      AtomRec a{};
      AtomRot z{};
      if (active) {
        a.x = in.x;
        a.y = in.y;
        a.z = in.z;
        a.occ = in.occ;
        a.bfac = in.bfac;
        a.log2occ = __log2f((float)a.occ);
        a.bl2e = (float)a.bfac * kLog2e;
        // the row recurrence's factors: e^{2 pi i z} and e^{-B G*33 / 2}
        sincospi(2.0 * a.z, &z.zs, &z.zc);
        z.rho = exp(-0.5 * a.bfac * P.gs[2]);
        z.zcf = (float)z.zc;
        z.zsf = (float)z.zs;
        z.rhof = (float)z.rho;
      }
      const uint64_t m = same_species(active, sp, nbits);
      const int below = lanes_below(m);
      const int pos = active ? mine[sp] + below : 0;
      wave_sync();
      if (active) {
        if (below == 0) mine[sp] = pos + __popcll(m);
        atoms[pos] = a;
        rot[pos] = z;
        orig[pos] = (int32_t)j;
      }
      wave_sync();
    }
#pragma unroll
    for (int u = 0; u < D; ++u) cur[u] = nxt[u];
  }
}

struct PackArgs {
  int32_t n_species;
  const double *frac;
  const int32_t *species;
  const double *occ;
  const double *bfac;
  const double *coeff;
  CoeffF *coeff_f;
  AtomRec *atoms;
  AtomRot *rot;
  int32_t *orig;
  SpeciesRun *runs;
  int32_t *run_count;
  int32_t *err;
};

// Atom packing alone, NW wavefronts per crystal.
template <int D, int NW>
__global__ __launch_bounds__(64 * NW) void k_atom_pack(const CrystalPlan *__restrict__ plan, int64_t n_c, PackArgs a) {
  extern __shared__ int32_t cursor[];  // NW x n_species
  pack_crystal<D, NW>(blockIdx.x, threadIdx.x & 63, cursor, plan, a.n_species, a.frac, a.species, a.occ, a.bfac, a.coeff,
               a.coeff_f, a.atoms, a.rot, a.orig, a.runs, a.run_count, a.err);
}

// Survivor count per enumeration chunk (at most kEnumRows rows), one
// wavefront per chunk (lane = row), four chunks per block.  The launch also
// packs the atoms (independent work) when its grid holds more blocks than
// the chunks need: the first blocks take four crystals each, one per
// wavefront, with n_species LDS cursors per wavefront; they come first so
// that their serial chains start with the counts rather than after them.
// With block_sums, each counting block also writes the sum of its four
// counts (block b of the counting blocks: chunks 4b .. 4b + 3).
__global__ __launch_bounds__(kThreads) void k_enum_count(const CrystalPlan *__restrict__ plan,
                                                         const EnumChunk *__restrict__ chunks,
                                                         int64_t n_chunks, int64_t n_c, double lambda,
                                                         int32_t *__restrict__ counts,
                                                         int64_t *__restrict__ block_sums, PackArgs pa) {
  const int64_t chunk_blocks = (n_chunks + kThreads / 64 - 1) / (kThreads / 64);
  const int64_t pack_blocks = (int64_t)gridDim.x - chunk_blocks;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  if (blockIdx.x < pack_blocks) {
    extern __shared__ int32_t cursors[];  // 4 x n_species
    const int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + wid;
    if (c < n_c)
      pack_crystal<1, 1>((int)c, lane, cursors + wid * pa.n_species, plan, pa.n_species, pa.frac, pa.species, pa.occ,
                   pa.bfac, pa.coeff, pa.coeff_f, pa.atoms, pa.rot, pa.orig, pa.runs, pa.run_count, pa.err);
    return;
  }
  const int64_t chunk = (int64_t)(blockIdx.x - pack_blocks) * (kThreads / 64) + wid;
  int n = 0;
  if (chunk < n_chunks) {
    const EnumChunk ch = chunks[chunk];
    const CrystalPlan &P = plan[ch.crystal];
    n = lane < ch.n_rows ? row_count(P, row_of(P, (int64_t)ch.row_begin + lane), lambda) : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d, 64);
    if (lane == 0) counts[chunk] = n;
  }
  if (block_sums) {
    // the block's four counts summed, for a fill that forms its own offsets
    __shared__ int32_t s_n[kThreads / 64];
    if (lane == 0) s_n[wid] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
#pragma unroll
      for (int v = 0; v < kThreads / 64; ++v) t += s_n[v];
      block_sums[blockIdx.x - pack_blocks] = t;
    }
  }
}

// Exclusive scan of the chunk counts and the crystal offsets in one block
// (batches with up to kOneBlockChunks enumeration chunks).
constexpr int kOneBlockChunks = 8192;
constexpr int kSelfChunks = 256;  // most chunks of one crystal for a fill that forms its own offsets
__global__ __launch_bounds__(1024) void k_enum_scan1(const CrystalPlan *__restrict__ plan, int64_t n_c,
                                                     int64_t n_chunks, const int32_t *__restrict__ counts,
                                                     int64_t *__restrict__ prefix, int64_t *__restrict__ refl_offset) {
  constexpr int PER = kOneBlockChunks / 1024;  // consecutive chunks per thread
  __shared__ int64_t s_pre[kOneBlockChunks + 1];
  __shared__ int64_t wsum[1024 / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // every load first: the thread's chunk counts and its crystals' first chunks
  // (n_c <= n_chunks <= kOneBlockChunks)
  int32_t v[PER], cb[PER];
  const int64_t i0 = (int64_t)threadIdx.x * PER;
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = i0 + u < n_chunks ? counts[i0 + u] : 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t c = threadIdx.x + (int64_t)u * 1024;
    cb[u] = c < n_c ? (int32_t)plan[c].enum_chunk_begin : 0;
  }
  int64_t sum = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) sum += v[u];
  int64_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t run = inc - sum, total = 0;
#pragma unroll
  for (int w = 0; w < 1024 / 64; ++w) {
    run += w < wid ? wsum[w] : 0;
    total += wsum[w];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (i0 + u < n_chunks) {
      s_pre[i0 + u] = run;
      prefix[i0 + u] = run;
    }
    run += v[u];
  }
  if (threadIdx.x == 0) {
    s_pre[n_chunks] = total;
    prefix[n_chunks] = total;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t c = threadIdx.x + (int64_t)u * 1024;
    if (c < n_c) refl_offset[c] = 2 * s_pre[cb[u]];
  }
  if (threadIdx.x == 0) refl_offset[n_c] = 2 * total;
}

__global__ void k_enum_offsets(const CrystalPlan *__restrict__ plan, int64_t n_c, int64_t n_chunks,
                               const int64_t *__restrict__ prefix, int64_t *__restrict__ refl_offset) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n_c) refl_offset[c] = 2 * prefix[plan[c].enum_chunk_begin];
  if (c == n_c) refl_offset[n_c] = 2 * prefix[n_chunks];
}

// Sum over a wavefront of one value per lane.
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// One wavefront per chunk (lane = row, for the chunk's first n_rows lanes),
// four chunks per block.  The chunk's rows are flattened into their candidate points in
// lexicographic order; the wavefront then takes the points 64 at a time, one
// per lane (a binary search over the rows' candidate offsets finds a point's
// row), tests them, ranks the survivors with a ballot and writes each with
// its Friedel mate: (h, k, l), q, 2theta and LP.
//
// Output positions come from the exclusive prefix P of the chunk counts: the
// crystal starts at 2 P(first chunk), holds 2 (P(end) - P(first)) reflections,
// and the chunk's survivors rank from P(chunk) - P(first).  Without SELF, P
// is a scanned array.  With SELF (at most kOneBlockChunks chunks, at most
// kSelfChunks per crystal) each block forms the values it needs from the
// counts themselves, so no scan launch sits between the count and the fill:
// the block sums the count launch's per-block sums before it (B = P(b0), b0
// its first chunk; both launches take kThreads / 64 chunks per block), and each
// wavefront sums the counts of [min(first, b0), end) in four parts, from
// which P(first) = B - sum[first, b0) + sum[b0, first), the crystal's count
// and the chunk's rank follow.  The wavefront at a crystal's first chunk
// writes refl_offset[c] = 2 P(first) (and refl_offset[n_c] for the last
// crystal): every crystal has at least one chunk.
template <bool SELF>
__global__ __launch_bounds__(kThreads) void k_enum_fill(const CrystalPlan *__restrict__ plan,
                                                        const EnumChunk *__restrict__ chunks,
                                                        int64_t n_chunks, const int64_t *__restrict__ prefix,
                                                        const int32_t *__restrict__ counts,
                                                        const int64_t *__restrict__ block_sums, int64_t n_c,
                                                        int64_t *__restrict__ refl_offset,
                                                        double lambda, int16_t *__restrict__ oh,
                                                        int16_t *__restrict__ ok, int16_t *__restrict__ ol,
                                                        double *__restrict__ oq, double *__restrict__ ott,
                                                        double *__restrict__ olp) {
  __shared__ int32_t s_off[kThreads / 64][kEnumRows + 1];  // candidate offsets of a wavefront's rows
  __shared__ int32_t s_lo[kThreads / 64][kEnumRows], s_h[kThreads / 64][kEnumRows], s_k[kThreads / 64][kEnumRows];
  __shared__ int64_t s_red[kThreads / 64];
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int64_t chunk = (int64_t)blockIdx.x * (kThreads / 64) + wid;
  const bool live = chunk < n_chunks;
  // wavefronts past the last chunk read the last one (they only take part in
  // the block's sum)
  const EnumChunk ch = chunks[live ? chunk : n_chunks - 1];
  const CrystalPlan &P = plan[ch.crystal];
  const int64_t first_chunk = P.enum_chunk_begin;
  int64_t c_begin, rh, rank0;
  if constexpr (SELF) {
    // every load first: the block sums before this block, then the counts
    // of [min(first, b0), end) (at most kSelfChunks + 3 of them)
    const int64_t b0 = (int64_t)blockIdx.x * (kThreads / 64), end = first_chunk + P.enum_chunks;
    const int64_t lo = min(first_chunk, b0);
    int64_t part = 0;
#pragma unroll
    for (int u = 0; u < kOneBlockChunks / (kThreads / 64) / kThreads; ++u) {
      const int64_t i = (int64_t)u * kThreads + threadIdx.x;
      if (i < (int64_t)blockIdx.x) part += block_sums[i];
    }
    int32_t before_b0 = 0, b0_to_first = 0, first_to_chunk = 0, crystal = 0;
#pragma unroll
    for (int u = 0; u < kSelfChunks / 64 + 1; ++u) {
      const int64_t i = lo + u * 64 + lane;
      if (i < end) {
        const int32_t v = counts[i];
        before_b0 += i < b0 ? v : 0;
        b0_to_first += i >= b0 && i < first_chunk ? v : 0;
        first_to_chunk += i >= first_chunk && i < chunk ? v : 0;
        crystal += i >= first_chunk ? v : 0;
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
    if (lane == 0) s_red[wid] = part;
    c_begin = wave_sum_i32(b0_to_first) - (int64_t)wave_sum_i32(before_b0);
    rank0 = wave_sum_i32(first_to_chunk);
    rh = wave_sum_i32(crystal);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kThreads / 64; ++v) c_begin += s_red[v];
    if (!live) return;
    if (chunk == first_chunk && lane == 0) {
      refl_offset[ch.crystal] = 2 * c_begin;
      if (ch.crystal == n_c - 1) refl_offset[n_c] = 2 * (c_begin + rh);
    }
  } else {
    if (!live) return;
    c_begin = prefix[first_chunk];
    rh = prefix[first_chunk + P.enum_chunks] - c_begin;  // positive-half count
    rank0 = prefix[chunk] - c_begin;
  }
  const int64_t seg = 2 * c_begin;  // crystal's first reflection
  int lo = 1, hi = 0;
  Row r{0, 0, 1, 0};
  if (lane < ch.n_rows) {
    r = row_of(P, (int64_t)ch.row_begin + lane);
    row_candidates(P, r, &lo, &hi);
  }
  const int nc = max(hi - lo + 1, 0);
  int inc = nc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  const int total = __shfl(inc, 63, 64);
  int32_t *off = s_off[wid];
  if (lane < kEnumRows) {
    off[lane] = inc - nc;
    s_lo[wid][lane] = lo;
    s_h[wid][lane] = r.h;
    s_k[wid][lane] = r.k;
  }
  if (lane == 0) off[kEnumRows] = total;
  wave_sync();
  int64_t rank = rank0;
  // four candidates per lane per round: their searches, tests and 2theta
  // are independent, so their latencies overlap
  constexpr int U = 4;
  for (int base = 0; base < total; base += 64 * U) {
    Hkl m[U];
    double q[U], tt[U];
    bool kp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ci = base + u * 64 + lane;
      m[u] = Hkl{0, 0, 0};
      q[u] = tt[u] = 0.0;
      kp[u] = false;
      if (ci < total) {
        int a = 0, b = kEnumRows - 1;  // last row whose offset is <= ci
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (off[mid] <= ci) a = mid; else b = mid - 1;
        }
        m[u] = Hkl{s_h[wid][a], s_k[wid][a], s_lo[wid][a] + (ci - off[a])};
        kp[u] = keep_point(P, m[u], lambda, true, &q[u], &tt[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t bal = __ballot(kp[u]);
      const int wrank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      const int64_t rk = rank + wrank;
      if (kp[u] && rk < rh) {  // rk < rh always: the count took the same decisions
        const int64_t pos = seg + rh + rk;
        const int64_t mate = seg + rh - 1 - rk;
        const double lp = lp_of_q(q[u], lambda);
        oh[pos] = (int16_t)m[u].h;
        ok[pos] = (int16_t)m[u].k;
        ol[pos] = (int16_t)m[u].l;
        oh[mate] = (int16_t)(-m[u].h);
        ok[mate] = (int16_t)(-m[u].k);
        ol[mate] = (int16_t)(-m[u].l);
        oq[pos] = q[u];
        oq[mate] = q[u];
        ott[pos] = tt[u];
        ott[mate] = tt[u];
        olp[pos] = lp;
        olp[mate] = lp;
      }
      rank += __popcll(bal);
    }
  }
}

}  // namespace

void launch_enumerate(const CrystalPlan *plan, int64_t n_c, const EnumChunk *chunks, int64_t n_chunks,
                      double lambda, int32_t *counts, int64_t *prefix, int64_t *scan_part, int16_t *h,
                      int16_t *k, int16_t *l, double *q, double *tt, double *lp, int64_t *refl_offset,
                      int32_t n_species, const double *frac, const int32_t *species, const double *occ,
                      const double *bfac, const double *coeff, CoeffF *coeff_f, AtomRec *atoms, AtomRot *rot,
                      int32_t *orig, SpeciesRun *runs, int32_t *run_count, int32_t *err, int64_t max_crystal_chunks,
                      int64_t max_crystal_atoms, hipStream_t s) {
  const PackArgs pa{n_species, frac, species, occ, bfac, coeff, coeff_f, atoms, rot, orig, runs, run_count, err};
  // the fill forms its own offsets when the counts are few and every crystal
  // has at least one chunk (so that one wavefront writes its offset)
  const bool self = n_chunks > 0 && n_chunks <= kOneBlockChunks && n_chunks >= n_c &&
                    max_crystal_chunks <= kSelfChunks;
  // the per-block sums of the counts take the scanned prefix's place
  int64_t *block_sums = self ? prefix : nullptr;
  // the packing rides along in the count launch while its cursors stay small
  // and its crystals small; otherwise a launch of its own, with four batches
  // of atom records in flight per wavefront
  const size_t fused_lds = (size_t)(kThreads / 64) * n_species * sizeof(int32_t);
  const bool fuse = n_chunks > 0 && fused_lds <= kFusedPackLds && max_crystal_atoms <= kFusedPackAtoms;
  if (!fuse && n_c > 0) {
    // eight wavefronts per crystal while their cursors fit in 64 KB of LDS
    // (measured on 2000-5000 atoms: 94 us with one, 44 with four, 35 with
    // eight, 56 with sixteen)
    const size_t lds8 = (size_t)8 * n_species * sizeof(int32_t);
    if (lds8 <= 65536)
      hipLaunchKernelGGL((k_atom_pack<4, 8>), dim3((unsigned)n_c), dim3(512), lds8, s, plan, n_c, pa);
    else
      hipLaunchKernelGGL((k_atom_pack<4, 1>), dim3((unsigned)n_c), dim3(64), (size_t)n_species * sizeof(int32_t), s,
                         plan, n_c, pa);
  }
  if (n_chunks > 0) {
    const int64_t chunk_blocks = (n_chunks + kThreads / 64 - 1) / (kThreads / 64);
    const int64_t pack_blocks = fuse ? (n_c + kThreads / 64 - 1) / (kThreads / 64) : 0;
    hipLaunchKernelGGL(k_enum_count, dim3((unsigned)(chunk_blocks + pack_blocks)), dim3(kThreads),
                       fuse ? fused_lds : 0, s, plan, chunks, n_chunks, n_c, lambda, counts, block_sums, pa);
  }
  if (!self) {
    if (n_chunks <= kOneBlockChunks) {
      hipLaunchKernelGGL(k_enum_scan1, dim3(1), dim3(1024), 0, s, plan, n_c, n_chunks, counts, prefix,
                         refl_offset);
    } else {
      launch_scan_i32(counts, n_chunks, nullptr, prefix, scan_part, s);
      hipLaunchKernelGGL(k_enum_offsets, dim3((unsigned)((n_c + 1 + 255) / 256)), dim3(256), 0, s, plan, n_c,
                         n_chunks, prefix, refl_offset);
    }
  }
  if (n_chunks > 0) {
    const dim3 grid((unsigned)((n_chunks + kThreads / 64 - 1) / (kThreads / 64)));
    if (self)
      hipLaunchKernelGGL(k_enum_fill<true>, grid, dim3(kThreads), 0, s, plan, chunks, n_chunks, prefix, counts,
                         block_sums, n_c, refl_offset, lambda, h, k, l, q, tt, lp);
    else
      hipLaunchKernelGGL(k_enum_fill<false>, grid, dim3(kThreads), 0, s, plan, chunks, n_chunks, prefix, counts,
                         block_sums, n_c, refl_offset, lambda, h, k, l, q, tt, lp);
  }
}

}  // namespace xrd
