// Sort of each crystal's reflections by (2theta, h, k, l) and the merge into
// peaks (paper, Section 2: merging of reflections within specified angular
// tolerances; grouping of reflections into peaks), fused per crystal.
//
// Sort: a classification pass splits the crystals by their reflection
// count; one launch then sorts each crystal of more than 2048 reflections with
// a 1024-thread block (in LDS up to 16384 reflections, through global memory
// beyond) and the smaller ones four to a block.  In LDS, a bucket sort with
// exactly monotone buckets, then each element's rank within its bucket on the
// full key (2theta, h, k, l), which removes the scatter's order dependence.
//
// Merge (anchor rule): walking the sorted order, a reflection joins the open
// peak while 2theta - 2theta(peak's first member) < tol.  A gap >= tol between
// neighbours always opens a peak, so the sorted list splits at such gaps into
// independent components; one thread walks each component with the anchor
// rule and flags peak starts.  A block scan of the flags numbers the peaks;
// the thread holding a peak's start sums its members' intensities in sorted
// order.  The block also takes the crystal's maximum and applies the relative
// threshold, leaving the crystal's peaks at its own reflection offset; a scan
// over crystals and a move kernel then pack them into CSR order and scale
// them to 0-100.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = kSortChunk / kThreads;  // 4
constexpr int64_t kPrefixCrystals = 4096;    // batches up to this size number their peaks in the move kernel

__device__ __forceinline__ int bin_of(const CrystalPlan &P, double tt) {
#pragma clang fp contract(off)
  const double x = floor((tt - P.tmin) * P.bin_scale);
  int b = x < 0.0 ? 0 : (x >= (double)(P.n_bins - 1) ? P.n_bins - 1 : (int)x);
  return b;
}

// Barrier that orders LDS accesses only: the wavefronts' global stores may
// still be in flight when it releases.  For phases whose threads exchange
// data through LDS and never read each other's global writes.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block barrier: LDS only (LDS_ONLY) or all memory.
template <bool LDS_ONLY>
__device__ __forceinline__ void block_barrier() {
  if constexpr (LDS_ONLY)
    lds_barrier();
  else
    __syncthreads();
}

// Exclusive scan of one int per thread over a group of T threads (``gt``:
// the thread's index in the group; ``wsum``: the group's T/64 ints of LDS).
// Its barriers are block-wide: every thread of the block calls it, as many
// times as the others.
template <int T, bool LDS_ONLY = false>
__device__ __forceinline__ int group_exclusive_scan(int v, int gt, int32_t *wsum, int *total) {
  const int lane = gt & 63, wid = gt >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  block_barrier<LDS_ONLY>();  // wsum may still be read from a previous call
  if (lane == 63) wsum[wid] = inc;
  block_barrier<LDS_ONLY>();
  int ex = inc - v, tot = 0;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) {
    ex += w < wid ? wsum[w] : 0;
    tot += wsum[w];
  }
  *total = tot;
  return ex;
}

// The same over the whole block (T threads).
template <int T, bool LDS_ONLY = false>
__device__ __forceinline__ int block_exclusive_scan(int v, int32_t *wsum, int *total) {
  return group_exclusive_scan<T, LDS_ONLY>(v, (int)threadIdx.x, wsum, total);
}

// Maximum of nonnegative doubles over a group (their bit patterns order like
// the values); block-wide barriers as above.
template <bool LDS_ONLY = false>
__device__ __forceinline__ double group_max_nonneg(double v, int gt, unsigned long long *slot) {
  // the wavefront's maximum first, so that one LDS atomic per wavefront
  // (not per thread) meets the shared slot
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  block_barrier<LDS_ONLY>();
  if (gt == 0) *slot = 0ull;
  block_barrier<LDS_ONLY>();
  if ((gt & 63) == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(v));
  block_barrier<LDS_ONLY>();
  return __longlong_as_double((long long)*slot);
}

// Where the fused merge leaves its results (null inten: sort only).
struct MergeOut {
  const double *inten;
  double tol, thr;
  int32_t *flags;       // [refl_cap] peak-start flags of the global-memory path
  double *t_tt, *t_i;   // a crystal's peaks at its reflection offset r0 + p
  int32_t *t_mult;
  int64_t *t_first;
  int32_t *pk_count;    // [n_c] peaks kept per crystal
  uint64_t *cmax;       // [n_c] bits of the crystal's largest peak intensity
  int64_t *perm;        // [refl_cap] global reflection index in sorted order
};

// Applies the relative threshold to peaks [0, np) of a crystal staged at r0
// (c < 0: the group has no crystal), compacting them in place (chunk by
// chunk: a chunk is read completely before any of it is written, and writes
// go to positions below the chunk's start or to its own slots), and records
// the count and maximum.  ``iters`` chunks of T are walked (>= np / T, the
// same for every group of the block, so that the barriers match).
template <int T>
__device__ void finish_crystal(const MergeOut &mo, int64_t c, int64_t r0, int np, double mx, int gt, int iters,
                               int32_t *wsum) {
  int kept = np;
  if (mo.thr > 0.0) {
    __syncthreads();  // the staged peaks of every thread are written
    const double cut = mo.thr * mx;
    kept = 0;
    for (int it = 0; it < iters; ++it) {
      const int p = it * T + gt;
      const bool live = p < np;
      double tt = 0.0, iv = 0.0;
      int32_t m = 0;
      int64_t f = 0;
      if (live) {
        tt = mo.t_tt[r0 + p];
        iv = mo.t_i[r0 + p];
        m = mo.t_mult[r0 + p];
        f = mo.t_first[r0 + p];
      }
      const bool keep = live && iv >= cut;
      int total;
      const int ex = group_exclusive_scan<T>(keep ? 1 : 0, gt, wsum, &total);  // its barriers order reads before writes
      if (keep) {
        mo.t_tt[r0 + kept + ex] = tt;
        mo.t_i[r0 + kept + ex] = iv;
        mo.t_mult[r0 + kept + ex] = m;
        mo.t_first[r0 + kept + ex] = f;
      }
      kept += total;
      __syncthreads();
    }
  }
  if (gt == 0 && c >= 0) {
    mo.pk_count[c] = kept;
    mo.cmax[c] = (uint64_t)__double_as_longlong(mx);
  }
}

// Global-memory sort and merge of one crystal by the whole block (T
// threads): the capacity-sized buckets of the plan, counted, scanned and
// filled with global atomics, then an insertion sort within buckets on
// (2theta, global index).  For crystals beyond the LDS sizes.
template <int T>
__device__ void sort_global(int64_t c, const CrystalPlan *__restrict__ plan, const int64_t *__restrict__ refl_offset,
                            const double *__restrict__ tt, double *__restrict__ skey, int32_t *__restrict__ sidx,
                            double *__restrict__ ent_key, int32_t *__restrict__ ent_idx, int32_t *__restrict__ bin_count,
                            int64_t *__restrict__ bin_start, const MergeOut &mo, int32_t *wsum,
                            unsigned long long *smax) {
  const bool merge = mo.inten != nullptr;
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  const int64_t R64 = r1 - r0;
  const int64_t e_base = r0 / 2;
  const CrystalPlan &P = plan[c];
  int total;
  const int64_t nb = P.n_bins;
  int32_t *__restrict__ bc = bin_count + P.bin_begin;
  int64_t *__restrict__ bs = bin_start + P.bin_begin;
  for (int64_t b = threadIdx.x; b < nb; b += T) bc[b] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < R64; i += T) atomicAdd(&bc[bin_of(P, tt[r0 + i])], 1);
  __syncthreads();
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += T) {
    const int64_t b = b0 + threadIdx.x;
    const int v = b < nb ? bc[b] : 0;
    const int ex = block_exclusive_scan<T>(v, wsum, &total);
    if (b < nb) bs[b] = carry + ex;
    carry += total;
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < R64; i += T) {
    const double t = tt[r0 + i];
    const int b = bin_of(P, t);
    const int64_t slot = r0 + bs[b] + atomicSub(&bc[b], 1) - 1;
    skey[slot] = t;
    sidx[slot] = (int32_t)(r0 + i);
  }
  __syncthreads();
  // ties by global index, which is lexicographic (h, k, l) order
  for (int64_t b = threadIdx.x; b < nb; b += T) {
    const int64_t s0 = r0 + bs[b], e0 = b + 1 < nb ? r0 + bs[b + 1] : r1;
    for (int64_t x = s0 + 1; x < e0; ++x) {
      const double kx = skey[x];
      const int32_t ix = sidx[x];
      int64_t j = x - 1;
      while (j >= s0) {
        const double kj = skey[j];
        const int32_t ij = sidx[j];
        if (!(kj > kx || (kj == kx && ij > ix))) break;
        skey[j + 1] = kj;
        sidx[j + 1] = ij;
        --j;
      }
      skey[j + 1] = kx;
      sidx[j + 1] = ix;
    }
  }
  __syncthreads();
  if (ent_key) {
    const int64_t mid = r0 + R64 / 2;
    int64_t done = 0;
    for (int64_t j0 = 0; j0 < R64; j0 += T) {
      const int64_t j = j0 + threadIdx.x;
      const bool f = j < R64 && sidx[r0 + j] >= mid;
      const int ex = block_exclusive_scan<T>(f ? 1 : 0, wsum, &total);
      if (f) {
        ent_key[e_base + done + ex] = skey[r0 + j];
        ent_idx[e_base + done + ex] = sidx[r0 + j];
      }
      done += total;
    }
  }
  if (merge) {
#pragma clang fp contract(off)
    // peak-start flags: one walker per component
    for (int64_t i = threadIdx.x; i < R64; i += T) {
      mo.perm[r0 + i] = sidx[r0 + i];
      const double ti = skey[r0 + i];
      if (i == 0 || ti - skey[r0 + i - 1] >= mo.tol) {
        mo.flags[r0 + i] = 1;
        double anchor = ti, prev = ti;
        for (int64_t j = i + 1; j < R64; ++j) {
          const double tj = skey[r0 + j];
          if (tj - prev >= mo.tol) break;
          const bool open = (tj - anchor) >= mo.tol;
          mo.flags[r0 + j] = open ? 1 : 0;
          if (open) anchor = tj;
          prev = tj;
        }
      }
    }
    __syncthreads();
    int64_t done = 0;
    double mx = 0.0;
    for (int64_t j0 = 0; j0 < R64; j0 += T) {
      const int64_t j = j0 + threadIdx.x;
      const bool f = j < R64 && mo.flags[r0 + j];
      const int ex = block_exclusive_scan<T>(f ? 1 : 0, wsum, &total);
      if (f) {
        const int64_t p = done + ex;
        double s = mo.inten[sidx[r0 + j]];
        int m = 1;
        for (int64_t x = j + 1; x < R64 && !mo.flags[r0 + x]; ++x) {
          s += mo.inten[sidx[r0 + x]];
          ++m;
        }
        mo.t_tt[r0 + p] = skey[r0 + j];
        mo.t_i[r0 + p] = s;
        mo.t_mult[r0 + p] = m;
        mo.t_first[r0 + p] = r0 + j;
        mx = fmax(mx, s);
      }
      done += total;
    }
    mx = group_max_nonneg(mx, (int)threadIdx.x, smax);
    finish_crystal<T>(mo, c, r0, (int)done, mx, (int)threadIdx.x, (int)((done + T - 1) / T), wsum);
  }
}

// ---- many-block global-memory sort ------------------------------------------
//
// The order and merge of sort_global, for crystals of capacity above
// kBigSort, spread over blocks of kBigChunk reflections, sorted positions or
// peak slots each, one launch per phase (a phase ends before the next reads
// its results, so no block waits on another), with no global atomics in the
// sort:
//   per-chunk histograms of nb 2theta buckets (monotone in 2theta, LDS
//   counters) -> a scan over the chunks of each bucket -> a scan over the
//   buckets -> scatter (each chunk's items to its ranges of their buckets,
//   ranked with LDS atomics) -> each bucket ordered in LDS on (2theta, global
//   index) by a bitonic network -> peak-start and entry flags with per-chunk counts ->
//   their scan per crystal -> write the entries and the peaks (each sum in
//   sorted order).
// The order on (2theta, global index) is total, so it is the one sort_global
// produces, whatever the bucketing.  With a relative threshold the peaks are
// staged in the upper half of the crystal's reflection slots (a crystal has
// at most R/2 peaks: both mates of a Friedel pair share 2theta bit for bit,
// so every peak holds both), then counted, scanned and compacted to its
// lower half.
constexpr int kBigThreads = 256;
constexpr int kBigPer = kBigChunk / kBigThreads;  // 16
// per-chunk counters (cnt) and their scans per crystal (off)
enum BigSlot { kSlotPeaks = 0, kSlotEntries = 1, kSlotKept = 2, kBigSlots = 3 };
constexpr int kWaveBucket = 512;   // items of a bucket ordered by one wavefront in LDS
constexpr int kBucketCap = 2048;   // ... by a block (the rare larger buckets); beyond, by insertion in place
constexpr int kOverBlocks = 64;    // blocks taking the buckets above kWaveBucket

struct BigArgs {
  const BigChunk *chunks;
  const CrystalPlan *plan;
  const int64_t *refl_offset;
  const double *tt;
  double *skey;
  int32_t *sidx;
  double *ent_key;  // null without Friedel pairing
  int32_t *ent_idx;
  int32_t *cnt;     // [kBigSlots n_big_chunks]
  int64_t *off;     // [kBigSlots n_big_chunks]
  int32_t *np;      // [n_c] peaks of a crystal
  int32_t *hist;    // per (chunk, bucket): count, then the exclusive scan over the chunks
  int64_t *boff;    // per (crystal, bucket): total, then the exclusive scan over the buckets
  int2 *over;       // (crystal list index, bucket) of the buckets above kWaveBucket items
  int32_t *n_over;  // their number
};

// The crystal of a chunk, if the many-block sort takes it (more than
// 2 kMidSort reflections; the others are sorted in LDS by the one-launch sort).
struct BigUnit {
  int64_t c, r0, R;
  int32_t chunk;
  int64_t slot;  // this chunk's first counter
  bool live;
};
__device__ __forceinline__ BigUnit big_unit(const BigArgs &a, const BigChunk &bc) {
  BigUnit u;
  u.c = bc.crystal;
  u.r0 = a.refl_offset[u.c];
  u.R = a.refl_offset[u.c + 1] - u.r0;
  u.chunk = bc.chunk;
  u.slot = (int64_t)kBigSlots * (bc.first + bc.chunk);
  u.live = u.R > 2 * (int64_t)kMidSort;
  return u;
}

// Sum of one int per thread over the block; ``red``: kBigThreads / 64 ints.
__device__ __forceinline__ int big_block_sum(int v, int32_t *red) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < kBigThreads / 64; ++w) t += red[w];
  return t;
}

// Block-wide ranks of the set lanes of one flag per thread: returns the
// number of set flags in lower threads and sets *total; ``red``: kBigThreads
// / 64 ints, free again on return.
__device__ __forceinline__ int big_block_rank(bool f, int32_t *red, int *total) {
  const uint64_t bal = __ballot(f);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = __popcll(bal);
  __syncthreads();
  int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
  int t = 0;
#pragma unroll
  for (int w = 0; w < kBigThreads / 64; ++w) {
    below += w < wid ? red[w] : 0;
    t += red[w];
  }
  __syncthreads();
  *total = t;
  return below;
}

// Bucket of 2theta t among nb (floor of an affine map with a positive slope,
// each step of which preserves order in IEEE arithmetic, so the bucket order
// never contradicts the key order).
__device__ __forceinline__ int big_bucket(const CrystalPlan &P, int nb, double t) {
#pragma clang fp contract(off)
  const double x = floor((t - P.tmin) * ((double)nb / (P.tmax - P.tmin)));
  return x < 0.0 ? 0 : (x >= (double)(nb - 1) ? nb - 1 : (int)x);
}

// Chunks holding reflections (the others take no part).
__device__ __forceinline__ int64_t big_filled_chunks(const BigUnit &u) { return (u.R + kBigChunk - 1) / kBigChunk; }

// Per chunk: its reflections' bucket counts (LDS atomics), written out.
__global__ __launch_bounds__(kBigThreads) void kb_hist(BigArgs a, uint64_t *__restrict__ cmax) {
  __shared__ int32_t h[kBigBucketsMax];
  const BigChunk bc = a.chunks[blockIdx.x];
  const BigUnit u = big_unit(a, bc);
  if (!u.live || u.chunk >= big_filled_chunks(u)) return;
  if (u.chunk == 0 && threadIdx.x == 0 && cmax) cmax[u.c] = 0ull;
  const CrystalPlan &P = a.plan[u.c];
  const int nb = bc.nb;
  for (int b = threadIdx.x; b < nb; b += kBigThreads) h[b] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)u.chunk * kBigChunk;
  for (int64_t i = i0 + threadIdx.x; i < min(i0 + kBigChunk, u.R); i += kBigThreads)
    atomicAdd(&h[big_bucket(P, nb, a.tt[u.r0 + i])], 1);
  __syncthreads();
  int32_t *__restrict__ out = a.hist + bc.hbase + (int64_t)u.chunk * nb;
  for (int b = threadIdx.x; b < nb; b += kBigThreads) out[b] = h[b];
}

// Per (crystal, bucket), a thread: the exclusive scan of the bucket's counts
// over the filled chunks (in place) and its total.
__global__ __launch_bounds__(kBigThreads) void kb_colscan(BigArgs a, const BigChunk *__restrict__ crystals) {
  const BigChunk bc = crystals[blockIdx.x];
  const BigUnit u = big_unit(a, bc);
  const int b = (int)blockIdx.y * kBigThreads + (int)threadIdx.x;
  if (!u.live || b >= bc.nb) return;
  const int64_t nk = big_filled_chunks(u);
  int32_t *__restrict__ col = a.hist + bc.hbase + b;
  int64_t run = 0;
  int64_t k = 0;
  for (; k + 8 <= nk; k += 8) {
    int32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = col[(k + q) * bc.nb];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      col[(k + q) * bc.nb] = (int32_t)run;
      run += v[q];
    }
  }
  for (; k < nk; ++k) {
    const int32_t v = col[k * bc.nb];
    col[k * bc.nb] = (int32_t)run;
    run += v;
  }
  a.boff[bc.bbase + b] = run;
}

// Per crystal: the exclusive scan of its bucket totals (in place), a
// thread's consecutive buckets at a time.
__global__ __launch_bounds__(kBigThreads) void kb_bscan(BigArgs a, const BigChunk *__restrict__ crystals) {
  __shared__ int32_t wsum[kBigThreads / 64];
  constexpr int PER = kBigBucketsMax / kBigThreads;  // 32
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_over = 0;
  const BigChunk bc = crystals[blockIdx.x];
  const BigUnit u = big_unit(a, bc);
  if (!u.live) return;
  int64_t *__restrict__ bo = a.boff + bc.bbase;
  const int b0 = (int)threadIdx.x * PER;
  int v[PER], s = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    v[q] = b0 + q < bc.nb ? (int)bo[b0 + q] : 0;
    s += v[q];
  }
  int total;
  int64_t o = block_exclusive_scan<kBigThreads>(s, wsum, &total);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (b0 + q < bc.nb) bo[b0 + q] = o;
    o += v[q];
  }
}

// Per chunk: each reflection to the next slot of its bucket's range for
// this chunk (the bucket's offset plus the chunk's column prefix), ranked
// with LDS atomics; the order inside a bucket is settled afterwards.
__global__ __launch_bounds__(kBigThreads) void kb_scatter(BigArgs a) {
  __shared__ int32_t cur[kBigBucketsMax];
  const BigChunk bc = a.chunks[blockIdx.x];
  const BigUnit u = big_unit(a, bc);
  if (!u.live || u.chunk >= big_filled_chunks(u)) return;
  const CrystalPlan &P = a.plan[u.c];
  const int nb = bc.nb;
  const int32_t *__restrict__ col = a.hist + bc.hbase + (int64_t)u.chunk * nb;
  // the chunk's reflections load while the cursors are set up, eight
  // cursors' loads in flight per thread at a time
  const int64_t i0 = (int64_t)u.chunk * kBigChunk;
  double t[kBigPer];
#pragma unroll
  for (int q = 0; q < kBigPer; ++q) {
    const int64_t i = i0 + q * kBigThreads + threadIdx.x;
    t[q] = i < u.R ? a.tt[u.r0 + i] : 0.0;
  }
  for (int b0 = threadIdx.x; b0 < nb; b0 += 8 * kBigThreads) {
    int64_t o[8];
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int b = b0 + q * kBigThreads;
      o[q] = b < nb ? a.boff[bc.bbase + b] : 0;
      c[q] = b < nb ? col[b] : 0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (b0 + q * kBigThreads < nb) cur[b0 + q * kBigThreads] = (int32_t)o[q] + c[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kBigPer; ++q) {
    const int64_t i = i0 + q * kBigThreads + threadIdx.x;
    if (i < u.R) {
      const int64_t slot = u.r0 + atomicAdd(&cur[big_bucket(P, nb, t[q])], 1);
      a.skey[slot] = t[q];
      a.sidx[slot] = (int32_t)(u.r0 + i);
    }
  }
}

// Ascending bitonic network over the n items at gk/gx, staged in LDS at
// sk/sx (room for the next power of two N >= n; padding sorts last) by the
// T threads ``t`` = 0 .. T-1 of a wavefront (T = 64) or of a block, which
// ``sync`` orders; pair p compares slot i (bit j clear) with i + j,
// ascending where bit k of i is clear.
template <int T, typename Sync>
__device__ __forceinline__ void bitonic_bucket(double *__restrict__ gk, int32_t *__restrict__ gx, int n, double *sk,
                                               int32_t *sx, int t, Sync sync) {
  int N = 2;
  while (N < n) N <<= 1;
  for (int i = t; i < N; i += T) {
    sk[i] = i < n ? gk[i] : __builtin_inf();
    sx[i] = i < n ? gx[i] : INT32_MAX;
  }
  sync();
  for (int k = 2; k <= N; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = t; p < N / 2; p += T) {
        const int i = 2 * p - (p & (j - 1)), l = i + j;
        const double ki = sk[i], kl = sk[l];
        const int32_t xi = sx[i], xl = sx[l];
        const bool gt = ki > kl || (ki == kl && xi > xl);
        if (gt == ((i & k) == 0)) {
          sk[i] = kl;
          sk[l] = ki;
          sx[i] = xl;
          sx[l] = xi;
        }
      }
      sync();
    }
  for (int i = t; i < n; i += T) {
    gk[i] = sk[i];
    gx[i] = sx[i];
  }
}

// The same ascending network over at most 64 E items in the registers of
// one wavefront: lane t holds slots E t .. E t + E - 1, slot i = E t + e in
// its e-th register (padding sorts last).  Pairs (i, i + j) with j < E are in
// one lane; for j >= E the partner sits at lane t ^ (j / E), register e, and
// each lane keeps the minimum or the maximum of the two by its slot's bits
// j and k.  No LDS and no barriers; (2theta, index) is a total order, so
// the result is the LDS network's.
template <int E>
__device__ __forceinline__ void bitonic_regs(double *__restrict__ gk, int32_t *__restrict__ gx, int n, int lane) {
  constexpr int N = 64 * E;
  double k[E];
  int32_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane * E + e;
    k[e] = i < n ? gk[i] : __builtin_inf();
    x[e] = i < n ? gx[i] : INT32_MAX;
  }
#pragma unroll
  for (int kk = 2; kk <= N; kk <<= 1)
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= E) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = lane * E + e;
          const double ko = __shfl_xor(k[e], j / E, 64);
          const int32_t xo = __shfl_xor(x[e], j / E, 64);
          const bool gt = k[e] > ko || (k[e] == ko && x[e] > xo);
          const bool keep_min = ((i & j) == 0) == ((i & kk) == 0);
          if (keep_min ? gt : !gt) {
            k[e] = ko;
            x[e] = xo;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (e & j) continue;
          const int f = e | j, i = lane * E + e;
          const bool gt = k[e] > k[f] || (k[e] == k[f] && x[e] > x[f]);
          if (gt == ((i & kk) == 0)) {
            const double tk = k[e];
            k[e] = k[f];
            k[f] = tk;
            const int32_t tx = x[e];
            x[e] = x[f];
            x[f] = tx;
          }
        }
      }
    }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = lane * E + e;
    if (i < n) {
      gk[i] = k[e];
      gx[i] = x[e];
    }
  }
}

__device__ __forceinline__ void big_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A bucket's range of sorted positions (relative to the crystal's r0).
__device__ __forceinline__ void big_bucket_range(const BigArgs &a, const BigChunk &bc, const BigUnit &u, int b,
                                                 int64_t *s0, int *n) {
  *s0 = a.boff[bc.bbase + b];
  const int64_t e0 = b + 1 < bc.nb ? a.boff[bc.bbase + b + 1] : u.R;
  *n = (int)(e0 - *s0);
}

// Per bucket of the batch, a wavefront (four buckets to a block): the
// bucket's items ordered in registers on (2theta, global index) and written
// back.  FLAT: the grid runs over the batch's buckets, crystal after
// crystal (a crystal's buckets start at its bbase), and each wavefront finds
// its crystal by a binary search over those starts (for batches of few
// large crystals of different sizes); otherwise grid (crystal, group of four
// buckets up to the largest count), blocks past a crystal's buckets ending
// at once (for many crystals, where the search would be long).  Buckets
// above kWaveBucket items, which the bucket sizing makes rare, are listed
// for kb_bsort_over.
template <bool FLAT>
__global__ __launch_bounds__(kBigThreads) void kb_bsort(BigArgs a, const BigChunk *__restrict__ crystals, int64_t n_big,
                                                        int64_t n_buckets) {
  static_assert(kWaveBucket == 512, "register networks of up to 8 items per lane");
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  int64_t lo;
  int b;
  if constexpr (FLAT) {
    const int64_t fb = (int64_t)blockIdx.x * (kBigThreads / 64) + wid;
    if (fb >= n_buckets) return;
    int64_t hi = n_big - 1;  // the last crystal whose buckets start at or before fb
    lo = 0;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (crystals[mid].bbase <= fb) lo = mid;
      else hi = mid - 1;
    }
    b = (int)(fb - crystals[lo].bbase);
  } else {
    lo = blockIdx.x;
    b = (int)blockIdx.y * (kBigThreads / 64) + wid;
  }
  const BigChunk bc = crystals[lo];
  const BigUnit u = big_unit(a, bc);
  if (!u.live || b >= bc.nb) return;
  int64_t s0;
  int n;
  big_bucket_range(a, bc, u, b, &s0, &n);
  if (n <= 1) return;
  if (n > kWaveBucket) {
    if (lane == 0) a.over[atomicAdd(a.n_over, 1)] = make_int2((int)lo, b);
    return;
  }
  double *gk = a.skey + u.r0 + s0;
  int32_t *gx = a.sidx + u.r0 + s0;
  if (n <= 64)
    bitonic_regs<1>(gk, gx, n, lane);
  else if (n <= 128)
    bitonic_regs<2>(gk, gx, n, lane);
  else if (n <= 256)
    bitonic_regs<4>(gk, gx, n, lane);
  else
    bitonic_regs<8>(gk, gx, n, lane);
}

// The listed buckets above kWaveBucket items, a block each in turn: the
// bitonic network in LDS up to kBucketCap items, an insertion sort in place
// by one thread beyond.
__global__ __launch_bounds__(kBigThreads) void kb_bsort_over(BigArgs a, const BigChunk *__restrict__ crystals) {
  __shared__ double sk[kBucketCap];
  __shared__ int32_t sx[kBucketCap];
  const int n_over = *a.n_over;
  for (int o = blockIdx.x; o < n_over; o += gridDim.x) {
    const int2 w = a.over[o];
    const BigChunk bc = crystals[w.x];
    const BigUnit u = big_unit(a, bc);
    int64_t s0;
    int n;
    big_bucket_range(a, bc, u, w.y, &s0, &n);
    double *__restrict__ gk = a.skey + u.r0 + s0;
    int32_t *__restrict__ gx = a.sidx + u.r0 + s0;
    if (n <= kBucketCap) {
      bitonic_bucket<kBigThreads>(gk, gx, n, sk, sx, (int)threadIdx.x, [] { __syncthreads(); });
      __syncthreads();  // the LDS is reused by the next bucket
      continue;
    }
    if (threadIdx.x == 0) {
      for (int xi = 1; xi < n; ++xi) {
        const double kx = gk[xi];
        const int32_t ix = gx[xi];
        int j = xi - 1;
        while (j >= 0 && (gk[j] > kx || (gk[j] == kx && gx[j] > ix))) {
          gk[j + 1] = gk[j];
          gx[j + 1] = gx[j];
          --j;
        }
        gk[j + 1] = kx;
        gx[j + 1] = ix;
      }
    }
  }
}

// Peak start at sorted position j: a gap >= tol before it, or the anchor
// rule walked from the start of its component (the last position at or
// before j with such a gap, or 0) up to j.  The same decisions as the one
// walker per component of sort_global, taken by each position for itself.
// A key equal to its predecessor's never opens a peak (tol > 0: the anchor
// is at most that key), which keeps shells of many equivalent reflections
// from walking.
__device__ __forceinline__ bool big_peak_start(const double *__restrict__ k, int64_t j, double tol) {
#pragma clang fp contract(off)
  if (j == 0 || k[j] - k[j - 1] >= tol) return true;
  if (k[j] == k[j - 1]) return false;
  int64_t s = j - 1;
  while (s > 0 && k[s] - k[s - 1] < tol) --s;
  double anchor = k[s];
  bool open = false;
  for (int64_t x = s + 1; x <= j; ++x) {
    open = (k[x] - anchor) >= tol;
    if (open) anchor = k[x];
  }
  return open;
}

// Per chunk of sorted positions: perm, the peak-start flags and the entry
// flags (the evaluated half: global index in the upper half of the
// crystal's slots), and their counts.
__global__ __launch_bounds__(kBigThreads) void kb_flags(BigArgs a, MergeOut mo) {
  __shared__ int32_t red[kBigThreads / 64];
  const BigUnit u = big_unit(a, a.chunks[blockIdx.x]);
  if (!u.live) return;
  const bool merge = mo.inten != nullptr;
  const int64_t mid = u.r0 + u.R / 2;
  const int64_t j0 = (int64_t)u.chunk * kBigChunk;
  int np = 0, ne = 0;
  for (int q = 0; q < kBigPer; ++q) {
    const int64_t j = j0 + q * kBigThreads + threadIdx.x;
    if (j >= u.R) break;
    const int32_t ix = a.sidx[u.r0 + j];
    ne += ix >= mid ? 1 : 0;
    if (merge) {
      mo.perm[u.r0 + j] = ix;
      const bool f = big_peak_start(a.skey + u.r0, j, mo.tol);
      mo.flags[u.r0 + j] = f ? 1 : 0;
      np += f ? 1 : 0;
    }
  }
  np = big_block_sum(np, red);
  ne = big_block_sum(ne, red);
  if (threadIdx.x == 0) {
    a.cnt[u.slot + kSlotPeaks] = np;
    a.cnt[u.slot + kSlotEntries] = ne;
  }
}

// Exclusive scan of a crystal's chunk counters ``k`` into off, one wavefront
// per crystal; returns the crystal's total.
__device__ int64_t big_scan_chunks(const BigArgs &a, const BigChunk &bc, int k) {
  const int lane = threadIdx.x & 63;
  int64_t carry = 0;
  for (int32_t i0 = 0; i0 < bc.n; i0 += 64) {
    const int32_t i = i0 + lane;
    const int64_t s = (int64_t)kBigSlots * ((int64_t)bc.first + i) + k;
    const int64_t v = i < bc.n ? a.cnt[s] : 0;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    if (i < bc.n) a.off[s] = carry + inc - v;
    carry += __shfl(inc, 63, 64);
  }
  return carry;
}

// Scans per crystal: the entry and peak counts, or the kept counts; with
// the peak counts the crystal's peak count (and, with no threshold to
// follow, its kept count), with the kept counts the latter.
enum BigScan { kScanFlags, kScanKept };
template <int WHICH>
__global__ __launch_bounds__(64) void kb_scan_counts(BigArgs a, const BigChunk *__restrict__ crystals, MergeOut mo) {
  const BigChunk bc = crystals[blockIdx.x];
  const BigUnit u = big_unit(a, bc);
  if (!u.live) return;
  if constexpr (WHICH == kScanFlags) {
    big_scan_chunks(a, bc, kSlotEntries);
    if (mo.inten == nullptr) return;
    const int64_t np = big_scan_chunks(a, bc, kSlotPeaks);
    if (threadIdx.x == 0) {
      a.np[u.c] = (int32_t)np;
      if (!(mo.thr > 0.0)) mo.pk_count[u.c] = (int32_t)np;
    }
  } else {
    const int64_t kept = big_scan_chunks(a, bc, kSlotKept);
    if (threadIdx.x == 0) mo.pk_count[u.c] = (int32_t)kept;
  }
}

// Per chunk of sorted positions: the entries at their ranks, and each peak
// (start, members' intensity sum in sorted order, multiplicity) at its
// number, staged at r0 + p (r0 + R/2 + p when a threshold follows); the
// crystal's largest peak intensity by one atomic per block.  Each window of
// kBigThreads positions gathers its intensities at once into LDS with the
// peak-start flags; a peak sums its members from there, in sorted order,
// and continues in global memory only past the window's end.
__global__ __launch_bounds__(kBigThreads) void kb_write(BigArgs a, MergeOut mo) {
  __shared__ int32_t red[kBigThreads / 64];
  __shared__ unsigned long long smax[1];
  __shared__ double s_v[kBigThreads];
  __shared__ int32_t s_f[kBigThreads];
  const BigUnit u = big_unit(a, a.chunks[blockIdx.x]);
  if (!u.live) return;
  const bool merge = mo.inten != nullptr, ent = a.ent_key != nullptr;
  const int64_t mid = u.r0 + u.R / 2;
  const int64_t j0 = (int64_t)u.chunk * kBigChunk;
  int64_t e = u.r0 / 2 + a.off[u.slot + kSlotEntries];
  int64_t p = a.off[u.slot + kSlotPeaks];
  const int64_t base = u.r0 + (mo.thr > 0.0 ? u.R / 2 : 0);
  double mx = 0.0;
  for (int q = 0; q < kBigPer; ++q) {
    const int64_t j = j0 + q * kBigThreads + threadIdx.x;
    if (j0 + q * kBigThreads >= u.R) break;  // the same for the whole block
    const bool live = j < u.R;
    const int32_t ix = live ? a.sidx[u.r0 + j] : 0;
    const bool fe = ent && live && ix >= mid;
    const bool fp = merge && live && mo.flags[u.r0 + j];
    int te, tp;
    const int re = big_block_rank(fe, red, &te);
    const int rp = big_block_rank(fp, red, &tp);
    if (fe) {
      a.ent_key[e + re] = a.skey[u.r0 + j];
      a.ent_idx[e + re] = ix;
    }
    if (merge) {
      // positions past the crystal stop a peak like a flag
      s_v[threadIdx.x] = live ? mo.inten[ix] : 0.0;
      s_f[threadIdx.x] = live ? (int32_t)mo.flags[u.r0 + j] : 1;
    }
    __syncthreads();
    if (fp) {
      double s = s_v[threadIdx.x];
      int m = 1;
      int t = (int)threadIdx.x + 1;
      for (; t < kBigThreads && !s_f[t]; ++t) {
        s += s_v[t];
        ++m;
      }
      if (t == kBigThreads)
        for (int64_t x = j0 + (int64_t)(q + 1) * kBigThreads; x < u.R && !mo.flags[u.r0 + x]; ++x) {
          s += mo.inten[a.sidx[u.r0 + x]];
          ++m;
        }
      mo.t_tt[base + p + rp] = a.skey[u.r0 + j];
      mo.t_i[base + p + rp] = s;
      mo.t_mult[base + p + rp] = m;
      mo.t_first[base + p + rp] = u.r0 + j;
      mx = fmax(mx, s);
    }
    e += te;
    p += tp;
    __syncthreads();  // s_v and s_f are written again by the next window
  }
  if (!merge) return;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mx = fmax(mx, __shfl_xor(mx, d, 64));
  if (threadIdx.x == 0) *smax = 0ull;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) atomicMax(smax, (unsigned long long)__double_as_longlong(mx));
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned long long *>(&mo.cmax[u.c]), *smax);
}

// Threshold, per chunk of staged peak slots: the kept peaks (I >= thr max),
// counted, then (after their scan) moved to r0 + rank.
template <bool MOVE>
__global__ __launch_bounds__(kBigThreads) void kb_keep(BigArgs a, MergeOut mo) {
  __shared__ int32_t red[kBigThreads / 64];
  const BigUnit u = big_unit(a, a.chunks[blockIdx.x]);
  if (!u.live) return;
  const int64_t np = a.np[u.c];
  const int64_t src = u.r0 + u.R / 2;
  const double cut = mo.thr * __longlong_as_double((long long)mo.cmax[u.c]);
  const int64_t k0 = (int64_t)u.chunk * kBigChunk;
  int nk = 0;
  int64_t d = u.r0 + (MOVE ? a.off[u.slot + kSlotKept] : 0);
  for (int q = 0; q < kBigPer; ++q) {
    const int64_t k = k0 + q * kBigThreads + threadIdx.x;
    if (k0 + q * kBigThreads >= np) break;  // the same for the whole block
    const double iv = k < np ? mo.t_i[src + k] : 0.0;
    const bool keep = k < np && iv >= cut;
    if constexpr (!MOVE) {
      nk += keep ? 1 : 0;
    } else {
      int t;
      const int r = big_block_rank(keep, red, &t);
      if (keep) {
        mo.t_tt[d + r] = mo.t_tt[src + k];
        mo.t_i[d + r] = iv;
        mo.t_mult[d + r] = mo.t_mult[src + k];
        mo.t_first[d + r] = mo.t_first[src + k];
      }
      d += t;
    }
  }
  if constexpr (!MOVE) {
    nk = big_block_sum(nk, red);
    if (threadIdx.x == 0) a.cnt[u.slot + kSlotKept] = nk;
  }
}

void big_sort(const SortArgs &s, const MergeOut &mo, hipStream_t st) {
  if (s.n_big_chunks <= 0) return;
  BigArgs a;
  a.chunks = s.big_chunks;
  a.plan = s.plan;
  a.refl_offset = s.refl_offset;
  a.tt = s.tt;
  a.skey = s.skey;
  a.sidx = s.sidx;
  a.ent_key = s.friedel ? s.ent_key : nullptr;
  a.ent_idx = s.friedel ? s.ent_idx : nullptr;
  a.cnt = s.big_cnt;
  a.off = s.big_off;
  a.np = s.big_np;
  a.hist = s.big_hist;
  a.boff = s.big_boff;
  a.over = s.big_over;
  a.n_over = reinterpret_cast<int32_t *>(s.big_over + s.big_buckets);
  const bool merge = mo.inten != nullptr;
  const dim3 g((unsigned)s.n_big_chunks), b(kBigThreads), gc((unsigned)s.n_big), w(64);
  const dim3 gcols((unsigned)s.n_big, (unsigned)((s.big_nb_max + kBigThreads - 1) / kBigThreads));
  // the bucket sort's grid: flat over the buckets for up to kFlatBig crystals
  constexpr int64_t kFlatBig = 64;
  const bool flat = s.n_big <= kFlatBig;
  const dim3 gbuckets = flat ? dim3((unsigned)((s.big_buckets + kBigThreads / 64 - 1) / (kBigThreads / 64)))
                             : dim3((unsigned)s.n_big, (unsigned)((s.big_nb_max + 3) / 4));
  hipLaunchKernelGGL(kb_hist, g, b, 0, st, a, merge ? mo.cmax : nullptr);
  hipLaunchKernelGGL(kb_colscan, gcols, b, 0, st, a, s.big_crystals);
  hipLaunchKernelGGL(kb_bscan, gc, b, 0, st, a, s.big_crystals);
  hipLaunchKernelGGL(kb_scatter, g, b, 0, st, a);
  if (flat)
    hipLaunchKernelGGL(kb_bsort<true>, gbuckets, b, 0, st, a, s.big_crystals, s.n_big, s.big_buckets);
  else
    hipLaunchKernelGGL(kb_bsort<false>, gbuckets, b, 0, st, a, s.big_crystals, s.n_big, s.big_buckets);
  hipLaunchKernelGGL(kb_bsort_over, dim3(kOverBlocks), b, 0, st, a, s.big_crystals);
  if (!merge && !a.ent_key) return;  // the sorted keys are the entries
  hipLaunchKernelGGL(kb_flags, g, b, 0, st, a, mo);
  hipLaunchKernelGGL(kb_scan_counts<kScanFlags>, gc, w, 0, st, a, s.big_crystals, mo);
  hipLaunchKernelGGL(kb_write, g, b, 0, st, a, mo);
  if (!merge || !(mo.thr > 0.0)) return;
  hipLaunchKernelGGL(kb_keep<false>, g, b, 0, st, a, mo);
  hipLaunchKernelGGL(kb_scan_counts<kScanKept>, gc, w, 0, st, a, s.big_crystals, mo);
  hipLaunchKernelGGL(kb_keep<true>, g, b, 0, st, a, mo);
}

// LDS sort and merge of one crystal of at most 2 CAP reflections by a group
// of T threads (``gt``: index in the group; c < 0: no crystal, the group only
// keeps step with the block's barriers).  The group's LDS: key[CAP],
// pos[CAP], cnt[CAP / 2], wsum[T / 64], one max slot.
//
// The crystal's Friedel-positive half is sorted (the mates follow from it
// exactly).  Buckets: H/2 of them, exactly monotone in 2theta (a product of
// nonnegative numbers, a subtraction, a product with a positive constant and
// floor each preserve order in IEEE arithmetic, so bucket order never
// contradicts key order and equal keys share a bucket); the cube of 2theta
// spreads the reflections evenly, their number growing about as the cube of
// the radius in reciprocal space.  Count with LDS atomics, scan, scatter with
// LDS atomics, then each element's rank within its bucket on (2theta bits,
// index).  The input is in lexicographic (h, k, l) order, so ordering ties by
// index orders them by (h, k, l); positive doubles order like their bit
// patterns.  The pair intensities (an entry and its mate) are loaded in input
// order, coalesced, and moved to their sorted slots in LDS (over the keys,
// once those are consumed), so the merge sums them without a gather; the
// peak starts are listed in LDS and one thread per peak sums and writes it.
//
// Outputs: without Friedel pairing, skey/sidx, the crystal's 2theta keys and
// global reflection indices in sorted order (the entries of the broadening);
// with it (ent_key non-null), the entries of the evaluated half (local index
// >= R/2) in sorted order, at entry positions starting at r0/2 (refl_offset
// values are even); with a merge, perm and the crystal's staged peaks.
template <int CAP, int T>
__device__ void sort_lds(int64_t c, int gt, uint64_t *key, uint16_t *pos, int32_t *cnt, int32_t *wsum,
                         unsigned long long *smax, const CrystalPlan *__restrict__ plan,
                         const int64_t *__restrict__ refl_offset, const double *__restrict__ tt,
                         double *__restrict__ skey, int32_t *__restrict__ sidx, double *__restrict__ ent_key,
                         int32_t *__restrict__ ent_idx, const MergeOut &mo) {
  constexpr int PER = CAP / T;
  const bool merge = mo.inten != nullptr;
  uint8_t *const fl = reinterpret_cast<uint8_t *>(cnt);
  double *const ival = reinterpret_cast<double *>(key);
  int64_t r0 = 0;
  int H = 0;
  double tmin = 0.0, tmax = 1.0;
  if (c >= 0) {
    r0 = refl_offset[c];
    H = (int)((refl_offset[c + 1] - r0) / 2);
    tmin = plan[c].tmin;
    tmax = plan[c].tmax;
  }
  const int64_t e_base = r0 / 2;
  int total;
  // Positives (local index H + i, i < H) and their mates (local H - 1 - i)
  // share 2theta bit for bit.  Sort the H positives by (2theta, i); a run of
  // equal keys [a, b] then expands, in (2theta, h, k, l) order, to the mates
  // of b, b-1, .., a (their local indices ascend that way) followed by the
  // positives a, .., b: full slots 2a + (b - j) and b + 1 + j for entry j.
  const int B = H / 2 > 1 ? H / 2 : 1;
  double lo, scale;
  {
#pragma clang fp contract(off)
    lo = tmin * tmin * tmin;
    const double span = tmax * tmax * tmax - lo;
    scale = span > 0.0 ? (double)B / span : 0.0;  // one bucket if the range's cubes coincide
  }
  auto bucket = [&](double t) {
#pragma clang fp contract(off)
    const double x = floor((t * t * t - lo) * scale);
    return x < 0.0 ? 0 : (x >= (double)(B - 1) ? B - 1 : (int)x);
  };
  for (int b = gt; b < B; b += T) cnt[b] = 0;
  // every thread's keys are loaded at once and kept in registers
  double tv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * T + gt;
    tv[u] = i < H ? tt[r0 + H + i] : tmin;
  }
  lds_barrier();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * T + gt;
    if (i < H) atomicAdd(&cnt[bucket(tv[u])], 1);
  }
  lds_barrier();
  // exclusive scan of the bucket counts: each thread owns a contiguous run
  {
    constexpr int per = (CAP / 2 + T - 1) / T;
    const int b0 = gt * per;
    int v[per], sum = 0;
#pragma unroll
    for (int u = 0; u < per; ++u) {
      v[u] = b0 + u < B ? cnt[b0 + u] : 0;
      sum += v[u];
    }
    int ex = group_exclusive_scan<T, true>(sum, gt, wsum, &total);
#pragma unroll
    for (int u = 0; u < per; ++u) {
      if (b0 + u < B) cnt[b0 + u] = ex;
      ex += v[u];
    }
  }
  lds_barrier();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * T + gt;
    if (i < H) {
      const int slot = atomicAdd(&cnt[bucket(tv[u])], 1);
      key[slot] = (uint64_t)__double_as_longlong(tv[u]);
      pos[slot] = (uint16_t)i;
    }
  }
  lds_barrier();
  // cnt[b] is now the end of bucket b, and its start is the end of bucket b - 1.
  // Order within buckets: every element counts the members of its bucket
  // that precede it in (2theta bits, index), all elements at once; then
  // each moves to its rank (all reads happen before the barrier, and the
  // ranks of a bucket are a permutation of its slots).
  int rk[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * T + gt;
    rk[u] = 0;
    if (i < H) {
      const uint64_t k = (uint64_t)__double_as_longlong(tv[u]);
      const int b = bucket(tv[u]);
      int r = b ? cnt[b - 1] : 0;
      for (int j = r, e0 = cnt[b]; j < e0; ++j) {
        const uint64_t kj = key[j];
        r += (kj < k || (kj == k && (int)pos[j] < i)) ? 1 : 0;
      }
      rk[u] = r;
    }
  }
  lds_barrier();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * T + gt;
    if (i < H) {
      key[rk[u]] = (uint64_t)__double_as_longlong(tv[u]);
      pos[rk[u]] = (uint16_t)i;
    }
  }
  lds_barrier();
  // entries (the evaluated half in 2theta order), the expanded full order
  // and, with a merge, the peak-start flags, in one pass: each entry's key
  // and its neighbours' are read once (a key run longer than one, rare,
  // reads further)
  for (int j = gt; j < H; j += T) {
    const uint64_t kj = key[j];
    const uint64_t kp = j > 0 ? key[j - 1] : 0ull;
    const uint64_t kn = j + 1 < H ? key[j + 1] : 0ull;
    const double tj = __longlong_as_double((long long)kj);
    const int p = pos[j];
    if (ent_key) {
      ent_key[e_base + j] = tj;
      ent_idx[e_base + j] = (int32_t)(r0 + H + p);
    }
    // the full order: as the merge's perm, and as the entries themselves
    // without Friedel pairing (skey/sidx are the entries then)
    if (!ent_key || merge) {
      int ga = j, gb = j;
      if (j > 0 && kp == kj) {
        ga = j - 1;
        while (ga > 0 && key[ga - 1] == kj) --ga;
      }
      if (j + 1 < H && kn == kj) {
        gb = j + 1;
        while (gb + 1 < H && key[gb + 1] == kj) ++gb;
      }
      const int fm = 2 * ga + (gb - j), fp = gb + 1 + j;
      const int64_t im = r0 + H - 1 - p, ip = r0 + H + p;
      if (!ent_key) {
        skey[r0 + fm] = tj;
        sidx[r0 + fm] = (int32_t)im;
        skey[r0 + fp] = tj;
        sidx[r0 + fp] = (int32_t)ip;
      }
      if (merge) {
        mo.perm[r0 + fm] = im;
        mo.perm[r0 + fp] = ip;
      }
    }
    if (merge) {
#pragma clang fp contract(off)
      // peak-start flags on the half (one byte per entry, in the bucket
      // table's space): one walker per component (a gap >= tol opens one);
      // mates never change the anchor walk, having the same 2theta as their
      // partner, and a peak start always begins a key run
      if (j == 0 || tj - __longlong_as_double((long long)kp) >= mo.tol) {
        fl[j] = 1;
        double anchor = tj, prev = tj;
        for (int m = j + 1; m < H; ++m) {
          const double tm = __longlong_as_double((long long)(m == j + 1 ? kn : key[m]));
          if (tm - prev >= mo.tol) break;
          const bool open = (tm - anchor) >= mo.tol;
          fl[m] = open ? 1 : 0;
          if (open) anchor = tm;
          prev = tm;
        }
      }
    }
  }
  if (merge) {
    // the pair intensities (an entry and its mate) in input order, coalesced
    double iv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = u * T + gt;
      iv[u] = i < H ? mo.inten[r0 + H - 1 - i] + mo.inten[r0 + H + i] : 0.0;
    }
    lds_barrier();  // every read of the keys is done: their space takes the pair intensities
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = u * T + gt;
      if (i < H) ival[rk[u]] = iv[u];
    }
    // number the peaks: each thread counts the starts in its run of PER
    // entries and lists them (in the sorted positions' space) at their numbers
    const int i0 = gt * PER;
    int ns = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) ns += (i0 + u < H && fl[i0 + u]) ? 1 : 0;
    int p = group_exclusive_scan<T, true>(ns, gt, wsum, &total);
    const int np = total;
    uint16_t *const pstart = pos;
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (i0 + u < H && fl[i0 + u]) pstart[p++] = (uint16_t)(i0 + u);
    // the starts and intensities in LDS, the entries' keys in global memory
    __syncthreads();
    // one thread per peak: its members' intensities summed in sorted order;
    // its 2theta is its first member's, the entry at its start (full-order
    // slot 2 start without Friedel pairing)
    double mx = 0.0;
    for (int q = gt; q < np; q += T) {
      const int a = pstart[q], e = q + 1 < np ? pstart[q + 1] : H;
      double sum = ival[a];
      for (int j = a + 1; j < e; ++j) sum += ival[j];
      mo.t_tt[r0 + q] = ent_key ? ent_key[e_base + a] : skey[r0 + 2 * a];
      mo.t_i[r0 + q] = sum;
      mo.t_mult[r0 + q] = 2 * (e - a);
      mo.t_first[r0 + q] = r0 + 2 * a;
      mx = fmax(mx, sum);
    }
    mx = group_max_nonneg<true>(mx, gt, smax);
    finish_crystal<T>(mo, c, r0, np, mx, gt, PER, wsum);
  }
}

// Exclusive scan of the per-crystal peak counts into peak_offset[0..n_c] by
// one block of 1024 threads, each taking kScanPer consecutive counts.
constexpr int kScanPer = 8;
__global__ __launch_bounds__(1024) void k_peak_scan(int64_t n_c, const int32_t *__restrict__ cnt,
                                                    int64_t *__restrict__ peak_offset) {
  __shared__ int32_t wsum[1024 / 64];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < n_c; c0 += 1024 * kScanPer) {
    const int64_t i0 = c0 + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
      v[u] = i0 + u < n_c ? cnt[i0 + u] : 0;
      sum += v[u];
    }
    int total;
    int ex = block_exclusive_scan<1024>(sum, wsum, &total);
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
      if (i0 + u < n_c) peak_offset[i0 + u] = carry + ex;
      ex += v[u];
    }
    carry += total;
  }
  if (threadIdx.x == 0) peak_offset[n_c] = carry;
}

// Sort (and merge) of every crystal in one launch of 1024-thread blocks.
// items[0, n_big) are the crystals whose capacity exceeds 2 kTinySort
// reflections: block b < n_big takes items[b] if it really has more than
// 2 kTinySort (the LDS sizes up to 2 CAPMAX reflections, the global-memory
// path beyond).  items[n_big, n_big + n_c) lists every crystal once more:
// each later block takes four of them, one per 256-thread group with a
// quarter of the LDS, and sorts those with at most 2 kTinySort.  Blocks
// with nothing to sort end at once.
template <int CAPMAX>
__global__ __launch_bounds__(1024, 8) void k_sort_merge(int64_t n_c, int64_t n_big, const int32_t *__restrict__ items,
                                                        const CrystalPlan *__restrict__ plan,
                                                        const int64_t *__restrict__ refl_offset,
                                                        const double *__restrict__ tt, double *__restrict__ skey,
                                                        int32_t *__restrict__ sidx, double *__restrict__ ent_key,
                                                        int32_t *__restrict__ ent_idx, int32_t *__restrict__ bin_count,
                                                        int64_t *__restrict__ bin_start, MergeOut mo) {
  static_assert(CAPMAX >= 4 * kTinySort, "four small crystals share the block's LDS");
  __shared__ uint64_t key[CAPMAX];
  __shared__ uint16_t pos[CAPMAX];
  __shared__ int32_t cnt[CAPMAX / 2];
  __shared__ int32_t wsum[1024 / 64];
  __shared__ unsigned long long smax[4];
  const int64_t blk = blockIdx.x;
  if (blk < n_big) {
    const int64_t c = items[blk];
    const int64_t R = refl_offset[c + 1] - refl_offset[c];
    if (R > 2 * (int64_t)CAPMAX) {
      // capacity above kBigSort: the many-block sort takes the crystal
      if (2 * plan[c].half_box <= kBigSort)
        sort_global<1024>(c, plan, refl_offset, tt, skey, sidx, ent_key, ent_idx, bin_count, bin_start, mo, wsum,
                          smax);
    }
    else if (R > 2 * kSmallSort)
      sort_lds<CAPMAX, 1024>(c, (int)threadIdx.x, key, pos, cnt, wsum, smax, plan, refl_offset, tt, skey, sidx,
                             ent_key, ent_idx, mo);
    else if (R > 2 * kTinySort)
      sort_lds<kSmallSort, 1024>(c, (int)threadIdx.x, key, pos, cnt, wsum, smax, plan, refl_offset, tt, skey, sidx,
                                 ent_key, ent_idx, mo);
  } else {
    // the four crystals of this block (every thread reads all four, so the
    // decision to skip is the block's)
    const int64_t first = (blk - n_big) * 4;
    int64_t cg[4];
    bool any = false;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      cg[g] = -1;
      if (first + g < n_c) {
        const int64_t c = items[n_big + first + g];
        if (refl_offset[c + 1] - refl_offset[c] <= 2 * kTinySort) cg[g] = c;
      }
      any = any || cg[g] >= 0;
    }
    if (any) {
      const int g = (int)(threadIdx.x >> 8);
      sort_lds<kTinySort, 256>(cg[g], (int)(threadIdx.x & 255), key + g * kTinySort, pos + g * kTinySort,
                               cnt + g * (kTinySort / 2), wsum + g * 4, smax + g, plan, refl_offset, tt, skey, sidx,
                               ent_key, ent_idx, mo);
    }
  }
}

// Sum over the block (kThreads threads) of one value per thread; ``red``
// holds kThreads / 64 values of LDS.  Every thread of the block must call it.
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *red) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  __syncthreads();  // red may still be read from a previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t t = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) t += red[w];
  return t;
}

// Packs each crystal's staged peaks at its peak offset and scales them:
// scaled = 100 I / max I of the crystal (0 when that maximum is 0).  One block
// per peak chunk (kSortChunk peak slots of one crystal, from a table of
// (crystal, chunk) pairs in which every crystal has at least its chunk 0).
// With ``prefix`` the block computes its crystal's offset itself, the sum of
// the counts of the crystals before it, and the block of a crystal's chunk 0
// writes it to peak_offset (block 0 also writes the total); otherwise the
// offsets come from a scan launched before.
__global__ __launch_bounds__(kThreads) void k_peak_move(const HChunk *__restrict__ chunks, int64_t n_c, bool prefix,
                                                        const int64_t *__restrict__ refl_offset,
                                                        int64_t *__restrict__ peak_offset, MergeOut mo,
                                                        double *__restrict__ pk_tt, double *__restrict__ pk_i,
                                                        double *__restrict__ pk_y, int32_t *__restrict__ pk_mult,
                                                        int64_t *__restrict__ pk_first) {
  __shared__ int64_t red[kThreads / 64];
  const HChunk ch = chunks[blockIdx.x];
  const int32_t c = ch.crystal;
  const int64_t k0 = (int64_t)ch.chunk * kSortChunk;
  // the crystal's values, loaded together
  const int np = mo.pk_count[c];
  const int64_t r0 = refl_offset[c];
  const double mx = __longlong_as_double((long long)mo.cmax[c]);
  // chunks past the crystal's peaks (the table covers its capacity) have
  // nothing to move; a crystal's chunk 0 still writes its offset and block 0
  // the total
  if (k0 >= np && ch.chunk != 0 && blockIdx.x != 0) return;
  // the chunk's staged peaks, loaded before the offset is known, so that their
  // latency overlaps the prefix sum's
  double tt[kPer], iv[kPer];
  int32_t m[kPer];
  int64_t f[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t k = k0 + u * kThreads + threadIdx.x;
    if (k < np) {
      tt[u] = mo.t_tt[r0 + k];
      iv[u] = mo.t_i[r0 + k];
      m[u] = mo.t_mult[r0 + k];
      f[u] = mo.t_first[r0 + k];
    }
  }
  int64_t o;
  if (prefix) {
    int64_t part = 0;
    for (int64_t i = threadIdx.x; i < c; i += kThreads) part += mo.pk_count[i];
    o = block_sum_i64(part, red);
    if (ch.chunk == 0 && threadIdx.x == 0) peak_offset[c] = o;
    if (blockIdx.x == 0) {
      int64_t all = 0;
      for (int64_t i = threadIdx.x; i < n_c; i += kThreads) all += mo.pk_count[i];
      all = block_sum_i64(all, red);
      if (threadIdx.x == 0) peak_offset[n_c] = all;
    }
  } else {
    o = peak_offset[c];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int64_t k = k0 + u * kThreads + threadIdx.x;
    if (k < np) {
      pk_tt[o + k] = tt[u];
      pk_i[o + k] = iv[u];
      pk_y[o + k] = mx > 0.0 ? 100.0 * iv[u] / mx : 0.0;
      pk_mult[o + k] = m[u];
      pk_first[o + k] = f[u];
    }
  }
}

MergeOut merge_out(const MergeArgs *m) {
  MergeOut mo{};
  if (!m) return mo;
  mo.inten = m->inten;
  mo.tol = m->tol;
  mo.thr = m->thr;
  mo.flags = m->flags;
  mo.t_tt = m->tmp_tt;
  mo.t_i = m->tmp_i;
  mo.t_mult = m->tmp_mult;
  mo.t_first = m->tmp_first;
  mo.pk_count = m->pk_count;
  mo.cmax = m->cmax;
  mo.perm = m->perm;
  return mo;
}

// The one sort launch: its grid covers every crystal that can exceed
// 2 kTinySort reflections (by capacity) plus every crystal again, four to a
// block.
void sort_kernels(const SortArgs &a, const MergeOut &mo, hipStream_t s) {
  if (a.n_c <= 0) return;
  double *ek = a.friedel ? a.ent_key : nullptr;
  int32_t *ei = a.friedel ? a.ent_idx : nullptr;
  const unsigned grid = (unsigned)(a.n_small + (a.n_c + 3) / 4);
  hipLaunchKernelGGL(k_sort_merge<kMidSort>, dim3(grid), dim3(1024), 0, s, a.n_c, a.n_small, a.items, a.plan,
                     a.refl_offset, a.tt, a.skey, a.sidx, ek, ei, a.bin_count, a.bin_start, mo);
  big_sort(a, mo, s);
}

}  // namespace

void launch_sort(const SortArgs &a, hipStream_t s) { sort_kernels(a, merge_out(nullptr), s); }

void launch_merge(const MergeArgs &a, hipStream_t s) {
  const SortArgs &o = a.sort;
  if (a.n_c <= 0) {
    launch_fill_u64(reinterpret_cast<uint64_t *>(a.peak_offset), 1, 0, s);
    return;
  }
  const MergeOut mo = merge_out(&a);
  sort_kernels(o, mo, s);
  // up to kPrefixCrystals crystals, each move block sums the counts before
  // its crystal (at most that many loads from L2) instead of waiting for a
  // one-block scan
  const bool prefix = a.n_c <= kPrefixCrystals;
  if (!prefix) hipLaunchKernelGGL(k_peak_scan, dim3(1), dim3(1024), 0, s, a.n_c, a.pk_count, a.peak_offset);
  hipLaunchKernelGGL(k_peak_move, dim3((unsigned)a.n_peak_chunks), dim3(kThreads), 0, s, a.peak_chunks, a.n_c, prefix,
                     o.refl_offset, a.peak_offset, mo, a.pk_tt, a.pk_i, a.pk_y, a.pk_mult, a.pk_first);
}

}  // namespace xrd
