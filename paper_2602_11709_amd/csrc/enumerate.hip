// Reciprocal-lattice enumeration inside the limiting sphere (paper, Section
// 2: generation of the reciprocal lattice points within the physically
// accessible sphere), with the per-reflection geometry q, 2theta and the
// Lorentz-polarisation factor.
//
// Each crystal's search box [-H,H]x[-K,K]x[-L,L] is split at the origin; only
// the points above it in lexicographic order are visited, since (h,k,l) and
// (-h,-k,-l) share q, 2theta and LP bit for bit.  Two passes over fixed-size
// chunks of that half box: count survivors per chunk, scan the counts, then
// recompute the test and write each survivor and its Friedel mate.  The
// output of a crystal is its full sphere shell in ascending (h, k, l) order:
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
constexpr int kPer = kEnumChunk / kThreads;  // 8
constexpr double kPi = 3.14159265358979323846;
constexpr size_t kFusedPackLds = 4096;  // largest cursor space the fused count-and-pack launch carries

struct Hkl {
  int h, k, l;
};

__device__ __forceinline__ Hkl decode(const CrystalPlan &P, int64_t p) {
  // linear index of the full box (h outermost); the origin is the centre.
  // The plan keeps boxes below 2^31 points, so 32-bit division suffices.
  const uint32_t nl = 2 * P.L + 1, nk = 2 * P.K + 1;
  const uint32_t i = (uint32_t)(P.half_box + 1 + p);
  Hkl r;
  const uint32_t t = i / nl;
  r.l = (int)(i - t * nl) - P.L;
  const uint32_t u = t / nk;
  r.k = (int)(t - u * nk) - P.K;
  r.h = (int)u - P.H;
  return r;
}

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

__device__ __forceinline__ bool keep(const CrystalPlan &P, int64_t p, double lambda, Hkl *m, double *q,
                                     double *tt) {
  if (p >= P.half_box) return false;
  *m = decode(P, p);
  *q = q_of(P, *m);
  if (*q < P.qlo || *q > P.qhi) return false;
  *tt = two_theta_of(*q, lambda);
  return *tt >= P.tmin && *tt <= P.tmax;
}

__device__ __forceinline__ double lp_of(double tt) {
#pragma clang fp contract(off)
  const double th = 0.5 * tt * (kPi / 180.0);
  double st, ct;
  sincos(th, &st, &ct);
  const double c2 = cos(2.0 * th);
  return (1.0 + c2 * c2) / (st * st * ct);
}

// ---- atom packing ----------------------------------------------------------
//
// The structure-factor kernels read each crystal's atoms grouped by species
// (so that the scattering factor is evaluated once per species and
// reflection), as 48-byte records.  One wavefront packs one crystal: species
// histogram in LDS, ascending-species runs, then a stable scatter (peeling one
// species per step with a ballot).  The wavefront works alone: it orders its
// LDS accesses with wavefront-scope fences, so several crystals can share a
// block.

constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ void pack_crystal(int c, int lane, int32_t *cursor, const CrystalPlan *__restrict__ plan,
                             int32_t n_species, const double *__restrict__ frac,
                             const int32_t *__restrict__ species, const double *__restrict__ occ,
                             const double *__restrict__ bfac, AtomRec *__restrict__ atoms,
                             int32_t *__restrict__ orig, SpeciesRun *__restrict__ runs,
                             int32_t *__restrict__ run_count, int32_t *__restrict__ err) {
  const CrystalPlan &P = plan[c];
  const int64_t a0 = P.atom_begin, a1 = P.atom_end;
  for (int t = lane; t < n_species; t += 64) cursor[t] = 0;
  wave_sync();
  for (int64_t j = a0 + lane; j < a1; j += 64) {
    int sp = species[j];
    if (sp < 0 || sp >= n_species) {
      atomicOr(err, 1);
      sp = 0;
    }
    atomicAdd(&cursor[sp], 1);
  }
  wave_sync();
  // ascending-species runs and cursors (exclusive scan of the histogram)
  int64_t running = a0;
  int nruns = 0;
  for (int t0 = 0; t0 < n_species; t0 += 64) {
    const int t = t0 + lane;
    const int v = t < n_species ? cursor[t] : 0;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    const int tot = __shfl(inc, 63, 64);
    const uint64_t nz = __ballot(v > 0);
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(nz >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nz, 0u));
    const int64_t start = running + inc - v;
    if (v > 0) {
      SpeciesRun r;
      r.begin = (int32_t)start;
      r.end = (int32_t)(start + v);
      r.species = t;
      r.local = nruns + rank;
      runs[P.run_begin + nruns + rank] = r;
    }
    if (t < n_species) cursor[t] = (int32_t)start;
    wave_sync();
    running += tot;
    nruns += __popcll(nz);
  }
  if (lane == 0) run_count[c] = nruns;
  for (int64_t base = a0; base < a1; base += 64) {
    const int64_t j = base + lane;
    bool active = j < a1;
    int sp = -1;
    if (active) {
      sp = species[j];
      if (sp < 0 || sp >= n_species) sp = 0;
    }
    while (true) {
      const uint64_t act = __ballot(active);
      if (act == 0) break;
      const int leader = __builtin_ctzll(act);
      const int t = __shfl(sp, leader, 64);
      const uint64_t m = __ballot(active && sp == t);
      const int base_pos = cursor[t];
      wave_sync();
      if (active && sp == t) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const int pos = base_pos + rank;
        AtomRec a;
        a.x = frac[3 * j];
        a.y = frac[3 * j + 1];
        a.z = frac[3 * j + 2];
        a.occ = occ[j];
        a.bfac = bfac[j];
        a.log2occ = __log2f((float)a.occ);
        a.bl2e = (float)a.bfac * kLog2e;
        atoms[pos] = a;
        orig[pos] = (int32_t)j;
        active = false;
      }
      if (lane == leader) cursor[t] = base_pos + __popcll(m);
      wave_sync();
    }
  }
}

struct PackArgs {
  int32_t n_species;
  const double *frac;
  const int32_t *species;
  const double *occ;
  const double *bfac;
  AtomRec *atoms;
  int32_t *orig;
  SpeciesRun *runs;
  int32_t *run_count;
  int32_t *err;
};

// Atom packing alone, one wavefront per crystal.
__global__ __launch_bounds__(64) void k_atom_pack(const CrystalPlan *__restrict__ plan, int64_t n_c, PackArgs a) {
  extern __shared__ int32_t cursor[];  // n_species
  pack_crystal(blockIdx.x, threadIdx.x, cursor, plan, a.n_species, a.frac, a.species, a.occ, a.bfac, a.atoms,
               a.orig, a.runs, a.run_count, a.err);
}

// Survivor count per enumeration chunk.  With pack_blocks > 0 the launch
// also packs the atoms (independent work): blocks from n_chunks on take four
// crystals each, one per wavefront, with n_species LDS cursors per wavefront.
__global__ __launch_bounds__(kThreads) void k_enum_count(const CrystalPlan *__restrict__ plan,
                                                         const int32_t *__restrict__ chunk_crystal,
                                                         int64_t n_chunks, int64_t n_c, double lambda,
                                                         int32_t *__restrict__ counts, PackArgs pa) {
  if (blockIdx.x >= n_chunks) {
    extern __shared__ int32_t cursors[];  // 4 x n_species
    const int wid = threadIdx.x >> 6;
    const int64_t c = (int64_t)(blockIdx.x - n_chunks) * (kThreads / 64) + wid;
    if (c < n_c)
      pack_crystal((int)c, threadIdx.x & 63, cursors + wid * pa.n_species, plan, pa.n_species, pa.frac, pa.species,
                   pa.occ, pa.bfac, pa.atoms, pa.orig, pa.runs, pa.run_count, pa.err);
    return;
  }
  const int chunk = blockIdx.x;
  const CrystalPlan &P = plan[chunk_crystal[chunk]];
  const int64_t p0 = (int64_t)(chunk - P.enum_chunk_begin) * kEnumChunk;
  int n = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    Hkl m;
    double q, tt;
    n += keep(P, p0 + u * kThreads + threadIdx.x, lambda, &m, &q, &tt) ? 1 : 0;
  }
  // block sum
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d, 64);
  __shared__ int ws[kThreads / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kThreads / 64; ++w) s += ws[w];
    counts[chunk] = s;
  }
}

// Exclusive scan of the chunk counts and the crystal offsets in one block
// (batches with up to kOneBlockChunks enumeration chunks).
constexpr int kOneBlockChunks = 8192;
__global__ __launch_bounds__(1024) void k_enum_scan1(const CrystalPlan *__restrict__ plan, int64_t n_c,
                                                     int64_t n_chunks, const int32_t *__restrict__ counts,
                                                     int64_t *__restrict__ prefix, int64_t *__restrict__ refl_offset) {
  __shared__ int64_t wsum[1024 / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < n_chunks; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < n_chunks ? counts[i] : 0;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    __syncthreads();
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 1024 / 64; ++w) {
      before += w < wid ? wsum[w] : 0;
      total += wsum[w];
    }
    if (i < n_chunks) prefix[i] = carry + before + inc - v;
    carry += total;
  }
  if (threadIdx.x == 0) prefix[n_chunks] = carry;
  __syncthreads();  // the block's prefix writes are visible to the whole block
  for (int64_t c = threadIdx.x; c <= n_c; c += 1024)
    refl_offset[c] = 2 * (c < n_c ? prefix[plan[c].enum_chunk_begin] : carry);
}

__global__ void k_enum_offsets(const CrystalPlan *__restrict__ plan, int64_t n_c, int64_t n_chunks,
                               const int64_t *__restrict__ prefix, int64_t *__restrict__ refl_offset) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n_c) refl_offset[c] = 2 * prefix[plan[c].enum_chunk_begin];
  if (c == n_c) refl_offset[n_c] = 2 * prefix[n_chunks];
}

__global__ __launch_bounds__(kThreads) void k_enum_fill(const CrystalPlan *__restrict__ plan,
                                                        const int32_t *__restrict__ chunk_crystal,
                                                        const int64_t *__restrict__ prefix, double lambda,
                                                        int16_t *__restrict__ oh, int16_t *__restrict__ ok,
                                                        int16_t *__restrict__ ol, double *__restrict__ oq,
                                                        double *__restrict__ ott, double *__restrict__ olp) {
  const int chunk = blockIdx.x;
  const CrystalPlan &P = plan[chunk_crystal[chunk]];
  const int64_t first_chunk = P.enum_chunk_begin;
  const int64_t c_begin = prefix[first_chunk];
  const int64_t rh = prefix[first_chunk + P.enum_chunks] - c_begin;  // positive-half count
  const int64_t seg = 2 * c_begin;                                     // crystal's first reflection
  int64_t rank = prefix[chunk] - c_begin;
  const int64_t p0 = (int64_t)(chunk - first_chunk) * kEnumChunk;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __shared__ int wcount[kPer][kThreads / 64];
  Hkl m[kPer];
  double q[kPer], tt[kPer];
  bool kp[kPer];
  int wrank[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    kp[u] = keep(P, p0 + u * kThreads + threadIdx.x, lambda, &m[u], &q[u], &tt[u]);
    const uint64_t b = __ballot(kp[u]);
    wrank[u] = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (lane == 0) wcount[u][wid] = __popcll(b);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      const int cnt = wcount[u][w];
      before += w < wid ? cnt : 0;
      total += cnt;
    }
    if (kp[u]) {
      const int64_t r = rank + before + wrank[u];
      const int64_t pos = seg + rh + r;
      const int64_t mate = seg + rh - 1 - r;
      const double lp = lp_of(tt[u]);
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
    rank += total;
  }
}

}  // namespace

void launch_enumerate(const CrystalPlan *plan, int64_t n_c, const int32_t *chunk_crystal, int64_t n_chunks,
                      double lambda, int32_t *counts, int64_t *prefix, int64_t *scan_part, int16_t *h,
                      int16_t *k, int16_t *l, double *q, double *tt, double *lp, int64_t *refl_offset,
                      int32_t n_species, const double *frac, const int32_t *species, const double *occ,
                      const double *bfac, AtomRec *atoms, int32_t *orig, SpeciesRun *runs, int32_t *run_count,
                      int32_t *err, hipStream_t s) {
  const PackArgs pa{n_species, frac, species, occ, bfac, atoms, orig, runs, run_count, err};
  // the packing rides along in the count launch while its cursors stay small
  const size_t fused_lds = (size_t)(kThreads / 64) * n_species * sizeof(int32_t);
  const bool fuse = n_chunks > 0 && fused_lds <= kFusedPackLds;
  if (!fuse && n_c > 0)
    hipLaunchKernelGGL(k_atom_pack, dim3((unsigned)n_c), dim3(64), (size_t)n_species * sizeof(int32_t), s, plan, n_c,
                       pa);
  if (n_chunks > 0) {
    const int64_t pack_blocks = fuse ? (n_c + kThreads / 64 - 1) / (kThreads / 64) : 0;
    hipLaunchKernelGGL(k_enum_count, dim3((unsigned)(n_chunks + pack_blocks)), dim3(kThreads),
                       fuse ? fused_lds : 0, s, plan, chunk_crystal, n_chunks, n_c, lambda, counts, pa);
  }
  if (n_chunks <= kOneBlockChunks) {
    hipLaunchKernelGGL(k_enum_scan1, dim3(1), dim3(1024), 0, s, plan, n_c, n_chunks, counts, prefix, refl_offset);
  } else {
    launch_scan_i32(counts, n_chunks, nullptr, prefix, scan_part, s);
    hipLaunchKernelGGL(k_enum_offsets, dim3((unsigned)((n_c + 1 + 255) / 256)), dim3(256), 0, s, plan, n_c, n_chunks,
                       prefix, refl_offset);
  }
  if (n_chunks > 0)
    hipLaunchKernelGGL(k_enum_fill, dim3((unsigned)n_chunks), dim3(kThreads), 0, s, plan, chunk_crystal, prefix,
                       lambda, h, k, l, q, tt, lp);
}

}  // namespace xrd
