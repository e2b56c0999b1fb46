// Families of symmetry-equivalent reflections in each merged peak (paper,
// Section 2: the grouping of symmetry-equivalent reflections is one of the
// steps moved to compiled code; Section 3's example output lists per peak its
// families, each with a multiplicity).
//
// Two reflections of a peak belong to one family when
//   indices rule: their absolute index values are equal as multisets, in the
//     form (h, k, l), or (h, k, -(h + k), l) on a hexagonal lattice;
//   lattice rule: a point operation M of the lattice (entries in {-1, 0, 1},
//     M^T G* M = G*) maps one onto the other, hkl -> M hkl.
// Both are class invariants of a key: the sorted absolute values, or the
// lexicographically largest image M hkl over the lattice's operations (an
// orbit has one largest member).  Members are taken in the peak's member
// order; a member whose key matches an existing family joins it, otherwise
// it opens the next family.  A family's label is its lexicographically
// largest member, its multiplicity the number of its members.
//
// One thread per peak: peaks hold a handful of members (a Friedel pair in a
// triclinic cell, up to 48 for a general cubic reflection), and a thread
// walks them in order with no synchronisation.  Up to kRegFam families of a
// peak live in registers (key, label, count); a peak with more families is
// redone by the general walk, which keeps the families in the peak's own
// stretch of the output arrays, in place: family f of a peak is created by a
// member at position >= f, so the slot holding the family's key (and later
// its label) never holds anything still needed.  Blocks follow the merge's
// peak chunks (crystal, 1024 peak slots), the expected-filled ones first.
#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int64_t kKeyBias = (int64_t)1 << 20;  // |M hkl| entries stay below 2^20

__device__ __forceinline__ void sort2(uint32_t &a, uint32_t &b) {
  const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

__device__ __forceinline__ uint64_t index_key(int h, int k, int l, bool hex) {
  uint32_t a = (uint32_t)abs(h), b = (uint32_t)abs(k), c = (uint32_t)abs(l), d = hex ? (uint32_t)abs(h + k) : 0u;
  // sorting network on four values (the fourth is 0 in the 3-index form, which
  // leaves the multiset comparison of the other three unchanged)
  sort2(a, b);
  sort2(c, d);
  sort2(a, c);
  sort2(b, d);
  sort2(b, c);
  return ((uint64_t)a << 48) | ((uint64_t)b << 32) | ((uint64_t)c << 16) | (uint64_t)d;
}

__device__ __forceinline__ uint64_t pack_hkl(int64_t h, int64_t k, int64_t l) {
  return ((uint64_t)(h + kKeyBias) << 42) | ((uint64_t)(k + kKeyBias) << 21) | (uint64_t)(l + kKeyBias);
}

__device__ __forceinline__ uint64_t lattice_key(int h, int k, int l, const FamOps &fo) {
  uint64_t best = 0;
  for (int o = 0; o < fo.n_ops; ++o) {
    const uint32_t m = fo.op[o];
    int v[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int m0 = (int)((m >> (6 * r)) & 3u) - 1, m1 = (int)((m >> (6 * r + 2)) & 3u) - 1,
                m2 = (int)((m >> (6 * r + 4)) & 3u) - 1;
      v[r] = m0 * h + m1 * k + m2 * l;
    }
    const uint64_t key = pack_hkl(v[0], v[1], v[2]);
    best = key > best ? key : best;
  }
  return best;
}

__device__ __forceinline__ uint64_t key_of(int h, int k, int l, bool lattice, const FamOps &fo) {
  return lattice ? lattice_key(h, k, l, fo) : index_key(h, k, l, fo.hex != 0);
}

constexpr int kRegFam = 4;

// The general walk over peak p's members (any number of families).
__device__ void families_in_place(int64_t p, const FamOps &fo, bool lattice, const int64_t *__restrict__ first,
                                  const int32_t *__restrict__ mult, const int64_t *__restrict__ perm,
                                  const int16_t *__restrict__ hh, const int16_t *__restrict__ kk,
                                  const int16_t *__restrict__ ll, int32_t *__restrict__ n_fam,
                                  int32_t *__restrict__ fam_of, int64_t *__restrict__ fam_label,
                                  int32_t *__restrict__ fam_mult) {
  const int64_t b = first[p];
  const int32_t m = mult[p];
  // pass 1: family of every member; keys of the open families at b + f
  int32_t nf = 0;
  for (int32_t i = 0; i < m; ++i) {
    const int64_t r = perm[b + i];
    const uint64_t key = key_of(hh[r], kk[r], ll[r], lattice, fo);
    int32_t f = 0;
    while (f < nf && (uint64_t)fam_label[b + f] != key) ++f;
    if (f == nf) {
      fam_label[b + nf] = (int64_t)key;
      fam_mult[b + nf] = 0;
      ++nf;
    }
    fam_of[b + i] = f;
    fam_mult[b + f] += 1;
  }
  // pass 2: labels (the keys are no longer needed)
  int32_t seen = 0;
  for (int32_t i = 0; i < m; ++i) {
    const int64_t r = perm[b + i];
    const int32_t f = fam_of[b + i];
    if (f == seen) {
      fam_label[b + f] = r;
      ++seen;
    } else {
      const int64_t c = fam_label[b + f];
      if (pack_hkl(hh[r], kk[r], ll[r]) > pack_hkl(hh[c], kk[c], ll[c])) fam_label[b + f] = r;
    }
  }
  n_fam[p] = nf;
}

__global__ void __launch_bounds__(kThreads) k_peak_families(
    const HChunk *__restrict__ chunks, const FamOps *__restrict__ fam_ops, const int64_t *__restrict__ peak_offset,
    const int64_t *__restrict__ first, const int32_t *__restrict__ mult, const int64_t *__restrict__ perm,
    const int16_t *__restrict__ hh, const int16_t *__restrict__ kk, const int16_t *__restrict__ ll, int rule,
    int32_t *__restrict__ n_fam, int32_t *__restrict__ fam_of, int64_t *__restrict__ fam_label,
    int32_t *__restrict__ fam_mult) {
  const HChunk ch = chunks[blockIdx.x];
  const int64_t p1 = peak_offset[ch.crystal + 1];
  const int64_t p0 = peak_offset[ch.crystal] + (int64_t)ch.chunk * kSortChunk;
  if (p0 >= p1) return;
  const FamOps &fo = fam_ops[ch.crystal];
  const bool lattice = rule == 1;
  for (int u = 0; u < kSortChunk / kThreads; ++u) {
    const int64_t p = p0 + u * kThreads + threadIdx.x;
    if (p >= p1) break;
    const int64_t b = first[p];
    const int32_t m = mult[p];
    uint64_t fk[kRegFam] = {}, lab[kRegFam] = {};
    int64_t li[kRegFam] = {};
    int32_t cnt[kRegFam] = {};
    int32_t nf = 0;
    bool spill = false;
    for (int32_t i = 0; i < m; ++i) {
      const int64_t r = perm[b + i];
      const int h = hh[r], k = kk[r], l = ll[r];
      const uint64_t key = key_of(h, k, l, lattice, fo);
      const uint64_t ph = pack_hkl(h, k, l);
      int32_t f = -1;
#pragma unroll
      for (int g = 0; g < kRegFam; ++g)
        if (f < 0 && g < nf && fk[g] == key) f = g;
      if (f < 0) {
        if (nf == kRegFam) {
          spill = true;
          break;
        }
        f = nf++;
#pragma unroll
        for (int g = 0; g < kRegFam; ++g)
          if (g == f) {
            fk[g] = key;
            lab[g] = ph;
            li[g] = r;
          }
      }
#pragma unroll
      for (int g = 0; g < kRegFam; ++g)
        if (g == f) {
          cnt[g] += 1;
          if (ph > lab[g]) {
            lab[g] = ph;
            li[g] = r;
          }
        }
      fam_of[b + i] = f;
    }
    if (spill) {
      families_in_place(p, fo, lattice, first, mult, perm, hh, kk, ll, n_fam, fam_of, fam_label, fam_mult);
      continue;
    }
#pragma unroll
    for (int g = 0; g < kRegFam; ++g)
      if (g < nf) {
        fam_label[b + g] = li[g];
        fam_mult[b + g] = cnt[g];
      }
    n_fam[p] = nf;
  }
}

}  // namespace

void launch_peak_families(const HChunk *chunks, int64_t n_chunks, const FamOps *fam_ops, const int64_t *peak_offset,
                          const int64_t *first, const int32_t *mult, const int64_t *perm, const int16_t *h,
                          const int16_t *k, const int16_t *l, int rule, int32_t *n_fam, int32_t *fam_of,
                          int64_t *fam_label, int32_t *fam_mult, hipStream_t s) {
  if (n_chunks <= 0) return;
  hipLaunchKernelGGL(k_peak_families, dim3((unsigned)n_chunks), dim3(kThreads), 0, s, chunks, fam_ops, peak_offset,
                     first, mult, perm, h, k, l, rule, n_fam, fam_of, fam_label, fam_mult);
}

}  // namespace xrd
