// Structure factors by a recurrence along reciprocal-lattice rows (the
// reciprocal-space partitioning the paper names as the way ahead, Section 5).
//
// A crystal's reflections are listed in lexicographic (h, k, l) order, so
// they form rows of fixed (h, k) and consecutive l (a row can break where the
// inner limit of the 2theta range cuts it).  Along a row the phase of atom j
// advances by 2 pi z_j per step and s^2 = q / 4 is a quadratic in l,
//   q(l) = G*33 l^2 + 2 (G*13 h + G*23 k) l + q(h, k, 0),
// so the weighted phasor of an atom obeys a two-term recurrence:
//   W(l) = occ e^{-B s^2(l)} e^{2 pi i (h x + k y + l z)},
//   W(l + 1) = W(l) T(l),  T(l) = r(l) e^{2 pi i z},  T(l + 1) = T(l) rho,
//   r(l) = e^{-B (q(l + 1) - q(l)) / 4},  rho = e^{-B G*33 / 2}.
// One lane takes a segment of at most kRecLen consecutive reflections of one
// row: per atom it evaluates W and T exactly at the segment's first
// reflection (the phase reduced mod 1, sin, cos and two exponentials) and
// steps the recurrence across the rest, a complex product and a real scaling
// per reflection instead of sin, cos and an exponential.  The segments tile
// each crystal's evaluated reflections in order (every row's run is cut into
// pieces of kRecLen from its first reflection), so every reflection is
// computed by exactly one lane, from an exact seed at most kRecLen - 1 steps
// back.
//
// The species factorisation, the per-species sums and their precision are
// those of the direct kernel: mixed precision sums each run of at most
// kAtomTile atoms of one species in single precision (the phase h x + k y +
// l z reduced mod 1 in double, sin/cos/exp2 and the recurrence in single) and
// adds the runs in double; the plain path does all of it in double.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int kAtomTile = 64;
constexpr int R = kRecLen;
constexpr double kLn2 = 0.69314718055994530942;

// Entries of a crystal: its evaluated reflections (the positive half under
// Friedel pairing, else every reflection) at global reflection indices
// first .. first + count - 1; entry e of crystal c sits at entry index
// base + e in the batch's entry space, base = r0 / 2 with pairing, else r0
// (so consecutive crystals' entries are contiguous).
struct Entries {
  int64_t first, count, base;
};
__device__ __forceinline__ Entries entries_of(const int64_t *__restrict__ refl_offset, int64_t c, bool friedel) {
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  Entries e;
  e.count = friedel ? (r1 - r0) / 2 : r1 - r0;
  e.first = r1 - e.count;
  e.base = friedel ? r0 / 2 : r0;
  return e;
}

__device__ __forceinline__ bool continues_row(const int16_t *__restrict__ h, const int16_t *__restrict__ k,
                                              const int16_t *__restrict__ l, int64_t i) {
  return h[i] == h[i - 1] && k[i] == k[i - 1] && l[i] == l[i - 1] + 1;
}

// Segment counts: one block per (crystal, kEntBlock entries); an entry that
// starts a run (its predecessor is in another row or not at l - 1) records
// ceil(run / kRecLen) segments, every other entry 0.  A run's length is
// the distance to the next run start: the block ballots its run starts into
// a kEntBlock-bit mask in LDS, and wavefront 0 measures how far the row of
// the block's last entry continues past the block (64 entries a round), for
// the last run that starts in the block.  Block 0 also records the batch's
// entry count for the scan.
__global__ __launch_bounds__(kThreads) void k_seg_count(const HChunk *__restrict__ eblocks, int64_t n_c,
                                                        const int64_t *__restrict__ refl_offset, bool friedel,
                                                        const int32_t *__restrict__ rec_of,
                                                        const int16_t *__restrict__ hh,
                                                        const int16_t *__restrict__ kk,
                                                        const int16_t *__restrict__ ll, int32_t *__restrict__ cnt,
                                                        int64_t *__restrict__ n_entries) {
  static_assert(kEntBlock == 4 * kThreads, "four entries per thread, one mask word per wavefront and slot");
  __shared__ uint64_t s_start[kEntBlock / 64];
  __shared__ int64_t s_cont;
  if (blockIdx.x == 0 && threadIdx.x == 0) n_entries[0] = friedel ? refl_offset[n_c] / 2 : refl_offset[n_c];
  const HChunk hk = eblocks[blockIdx.x];
  const Entries en = entries_of(refl_offset, hk.crystal, friedel);
  const bool rec = rec_of[hk.crystal] != 0;  // other crystals get no segments
  const int64_t e0 = (int64_t)hk.chunk * kEntBlock;
  const int64_t e1 = min(e0 + (int64_t)kEntBlock, en.count);
  if (e0 >= e1) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (!rec) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) cnt[en.base + e] = 0;
    return;
  }
  // entry e0 + 256 u + t: slot u of thread t, mask word 4 u + (t / 64)
  bool st[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t e = e0 + u * kThreads + threadIdx.x;
    st[u] = e < e1 && (e == 0 || !continues_row(hh, kk, ll, en.first + e));
    const uint64_t b = __ballot(st[u]);
    if (lane == 0) s_start[4 * u + wid] = b;
  }
  if (wid == 0) {
    // entries past the block that continue the row of its last entry
    int64_t c = 0;
    for (int64_t j0 = e1;; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool more = j < en.count && continues_row(hh, kk, ll, en.first + j);
      const uint64_t b = __ballot(more);
      if (b == ~0ull) {
        c += 64;
        continue;
      }
      c += __builtin_ctzll(~b);
      break;
    }
    if (lane == 0) s_cont = c;
  }
  __syncthreads();
  const int nb = (int)(e1 - e0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int p = u * kThreads + (int)threadIdx.x;  // position in the block
    if (p >= nb) continue;
    int32_t n = 0;
    if (st[u]) {
      // the next run start after p in the mask, else the block's end plus
      // the continuation
      int64_t len = -1;
      int w = p >> 6;
      uint64_t m = (p & 63) == 63 ? 0ull : s_start[w] & (~0ull << ((p & 63) + 1));
      while (true) {
        if (m != 0ull) {
          len = (int64_t)(64 * w + __builtin_ctzll(m)) - p;
          break;
        }
        if (++w >= kEntBlock / 64) break;
        m = s_start[w];
      }
      if (len < 0 || p + len > nb) len = (int64_t)nb - p + s_cont;
      n = (int32_t)((len + R - 1) / R);
    }
    cnt[en.base + e0 + p] = n;
  }
}

// Segment starts: each run start writes the global reflection index of its
// segments' first reflections at their global segment indices (the
// exclusive scan of the counts).
__global__ __launch_bounds__(kThreads) void k_seg_write(const HChunk *__restrict__ eblocks,
                                                        const int64_t *__restrict__ refl_offset, bool friedel,
                                                        const int32_t *__restrict__ cnt,
                                                        const int64_t *__restrict__ seg_index,
                                                        int32_t *__restrict__ seg_start) {
  const HChunk hk = eblocks[blockIdx.x];
  const Entries en = entries_of(refl_offset, hk.crystal, friedel);
  const int64_t e0 = (int64_t)hk.chunk * kEntBlock;
  for (int64_t e = e0 + threadIdx.x; e < min(e0 + (int64_t)kEntBlock, en.count); e += kThreads) {
    const int n = cnt[en.base + e];
    const int64_t s = seg_index[en.base + e];
    for (int j = 0; j < n; ++j) seg_start[s + j] = (int32_t)(en.first + e + (int64_t)j * R);
  }
}

// Which part of the batch a wavefront takes (as in the direct kernel): the
// first n_heavy items take a block each, its four wavefronts splitting the
// crystal's atoms into contiguous quarters; the rest go four to a block.
struct WaveWork {
  int64_t item;
  int part, nparts;
  bool heavy;
};
__device__ __forceinline__ WaveWork wave_work(int64_t n_heavy) {
  WaveWork w;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  w.heavy = blockIdx.x < n_heavy;
  if (w.heavy) {
    w.item = blockIdx.x;
    w.part = wid;
    w.nparts = kThreads / 64;
  } else {
    w.item = n_heavy + (int64_t)(blockIdx.x - n_heavy) * (kThreads / 64) + wid;
    w.part = 0;
    w.nparts = 1;
  }
  return w;
}

__device__ __forceinline__ float fsc_df_f32(const CoeffF &cf, float s2, float *df) {
  float a = cf.c, d = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float e = __builtin_amdgcn_exp2f(cf.nbl[i] * s2);
    a = fmaf(cf.a[i], e, a);
    d = fmaf(cf.nab[i], e, d);
  }
  *df = d;
  return a;
}

__device__ __forceinline__ double fsc_df_f64(const double *__restrict__ c9, double s2, double *df) {
  double a = c9[8], d = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double e = exp(-c9[4 + i] * s2);
    a = fma(c9[i], e, a);
    d = fma(-c9[i] * c9[4 + i], e, d);
  }
  *df = d;
  return a;
}

template <bool MIXED>
__device__ __forceinline__ void store_derivs(void *cache, int64_t i, double A, double B, double dA, double dB) {
  if constexpr (MIXED)
    reinterpret_cast<float4 *>(cache)[i] = make_float4((float)A, (float)B, (float)dA, (float)dB);
  else
    reinterpret_cast<double4 *>(cache)[i] = make_double4(A, B, dA, dB);
}

// Sums of one wavefront's segments over its atoms [wa, wb) of the crystal's
// runs: for each of the lane's kRecLen reflections (A, B) and, with DERIV,
// (dA, dB)/ds^2, per run t
//   S_t = sum_{j in t} W_j,  S'_t = sum_{j in t} (-B_j) W_j,
//   A + iB += f_t S_t,  d(A + iB)/ds^2 += f'_t S_t + f_t S'_t.
// Mixed: S_t, S'_t in single precision over chunks of kAtomTile atoms (S'_t
// carrying B log2(e) W, the factor -ln 2 joining f), added in double.
template <bool MIXED, bool DERIV>
__device__ __forceinline__ void rec_sums(const SpeciesRun *__restrict__ cr, int nr, int wa, int wb,
                                         const AtomRec *__restrict__ atoms, const AtomRot *__restrict__ rot,
                                         const double *__restrict__ coeff, const CoeffF *__restrict__ coeff_f,
                                         double h, double k, double l0, const double (&s2d)[R], double dq0,
                                         double (&acc)[DERIV ? 4 : 2][R]) {
#pragma unroll
  for (int v = 0; v < (DERIV ? 4 : 2); ++v)
#pragma unroll
    for (int u = 0; u < R; ++u) acc[v][u] = 0.0;
  if constexpr (MIXED) {
    float s2[R];
#pragma unroll
    for (int u = 0; u < R; ++u) s2[u] = (float)s2d[u];
    const float s20 = s2[0], qstep = (float)(0.25 * dq0);
    for (int ir = 0; ir < nr; ++ir) {
      const SpeciesRun run = cr[ir];
      const int rb = max(run.begin, wa), re = min(run.end, wb);
      if (rb >= re) continue;
      const CoeffF cf = coeff_f[run.species];
      float f[R], df[R];
#pragma unroll
      for (int u = 0; u < R; ++u) f[u] = fsc_df_f32(cf, s2[u], &df[u]);
      for (int j0 = rb; j0 < re; j0 += kAtomTile) {
        const int j1 = min(j0 + kAtomTile, re);
        float pa[R], pb[R], qa[R], qb[R];
#pragma unroll
        for (int u = 0; u < R; ++u) pa[u] = pb[u] = qa[u] = qb[u] = 0.f;
        // the seed of atom a at the segment's first reflection, then the
        // recurrence across the segment
        auto walk = [&](const AtomRec &a, const AtomRot &z) {
          const double t = fma(h, a.x, fma(k, a.y, l0 * a.z));
          const float rho = (float)__builtin_amdgcn_fract(t);
          const float sn = __builtin_amdgcn_sinf(rho);
          const float cs = __builtin_amdgcn_cosf(rho);
          const float d0 = __builtin_amdgcn_exp2f(fmaf(-a.bl2e, s20, a.log2occ));
          const float r0 = __builtin_amdgcn_exp2f(-a.bl2e * qstep);
          float wr = d0 * cs, wi = d0 * sn;
          float tr = r0 * z.zcf, ti = r0 * z.zsf;
#pragma unroll
          for (int u = 0; u < R; ++u) {
            pa[u] += wr;
            pb[u] += wi;
            if constexpr (DERIV) {
              qa[u] = fmaf(a.bl2e, wr, qa[u]);
              qb[u] = fmaf(a.bl2e, wi, qb[u]);
            }
            if (u + 1 < R) {
              const float nr_ = fmaf(wr, tr, -wi * ti);
              const float ni_ = fmaf(wr, ti, wi * tr);
              wr = nr_;
              wi = ni_;
              tr *= z.rhof;
              ti *= z.rhof;
            }
          }
        };
        int j = j0;
        for (; j + 2 <= j1; j += 2) {
          const AtomRec a0 = atoms[j], a1 = atoms[j + 1];
          const AtomRot z0 = rot[j], z1 = rot[j + 1];
          walk(a0, z0);
          walk(a1, z1);
        }
        for (; j < j1; ++j) walk(atoms[j], rot[j]);
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const double fu = f[u];
          acc[0][u] = fma(fu, (double)pa[u], acc[0][u]);
          acc[1][u] = fma(fu, (double)pb[u], acc[1][u]);
          if constexpr (DERIV) {
            const double fq = -kLn2 * fu, dfu = df[u];
            acc[2][u] = fma(dfu, (double)pa[u], fma(fq, (double)qa[u], acc[2][u]));
            acc[3][u] = fma(dfu, (double)pb[u], fma(fq, (double)qb[u], acc[3][u]));
          }
        }
      }
    }
  } else {
    const double s20 = s2d[0], qstep = 0.25 * dq0;
    for (int ir = 0; ir < nr; ++ir) {
      const SpeciesRun run = cr[ir];
      const int rb = max(run.begin, wa), re = min(run.end, wb);
      if (rb >= re) continue;
      const double *c9 = coeff + 9 * run.species;
      double f[R], df[R], pa[R], pb[R], qa[R], qb[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        f[u] = fsc_df_f64(c9, s2d[u], &df[u]);
        pa[u] = pb[u] = qa[u] = qb[u] = 0.0;
      }
      for (int j = rb; j < re; ++j) {
        const AtomRec a = atoms[j];
        const AtomRot z = rot[j];
        const double t = fma(h, a.x, fma(k, a.y, l0 * a.z));
        const double rho = t - rint(t);
        double sn, cs;
        sincospi(2.0 * rho, &sn, &cs);
        const double d0 = a.occ * exp(-a.bfac * s20);
        const double r0 = exp(-a.bfac * qstep);
        double wr = d0 * cs, wi = d0 * sn;
        double tr = r0 * z.zc, ti = r0 * z.zs;
        const double nb = -a.bfac;
#pragma unroll
        for (int u = 0; u < R; ++u) {
          pa[u] += wr;
          pb[u] += wi;
          if constexpr (DERIV) {
            qa[u] = fma(nb, wr, qa[u]);
            qb[u] = fma(nb, wi, qb[u]);
          }
          if (u + 1 < R) {
            const double nr_ = fma(wr, tr, -wi * ti);
            const double ni_ = fma(wr, ti, wi * tr);
            wr = nr_;
            wi = ni_;
            tr *= z.rho;
            ti *= z.rho;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        acc[0][u] = fma(f[u], pa[u], acc[0][u]);
        acc[1][u] = fma(f[u], pb[u], acc[1][u]);
        if constexpr (DERIV) {
          acc[2][u] += df[u] * pa[u] + f[u] * qa[u];
          acc[3][u] += df[u] * pb[u] + f[u] * qb[u];
        }
      }
    }
  }
}

// One item = up to 64 segments of one crystal (one per lane).  Light items
// take a wavefront; heavy ones a block whose four wavefronts sum contiguous
// quarters of the atoms, their sums added in LDS in a fixed order
// (((w3 + w2) + w1) + w0).
template <bool MIXED, bool FRIEDEL, bool DERIV>
__global__ __launch_bounds__(kThreads) void k_sf_rec(
    const SfItem *__restrict__ items, int64_t n_items, int64_t n_heavy, const CrystalPlan *__restrict__ plan,
    const int64_t *__restrict__ refl_offset, const int64_t *__restrict__ seg_index,
    const int32_t *__restrict__ seg_start, const int16_t *__restrict__ hh, const int16_t *__restrict__ kk,
    const int16_t *__restrict__ ll, const double *__restrict__ qq, const double *__restrict__ lpp,
    const AtomRec *__restrict__ atoms, const AtomRot *__restrict__ rot, const SpeciesRun *__restrict__ runs,
    const int32_t *__restrict__ run_count, const double *__restrict__ coeff, const CoeffF *__restrict__ coeff_f,
    void *__restrict__ Aout, void *__restrict__ Bout, double *__restrict__ Iout, void *__restrict__ cache) {
  constexpr int V = DERIV ? 4 : 2;
  __shared__ double s_red[V * R * 64];
  const WaveWork ww = wave_work(n_heavy);
  if (ww.item >= n_items) return;  // light blocks only: a heavy block's item always exists
  const SfItem it = items[ww.item];
  const Entries en = entries_of(refl_offset, it.crystal, FRIEDEL);
  const int64_t sb = seg_index[en.base], se = seg_index[en.base + en.count];
  // a tail item walks the crystal's segment tiles from its first one on
  auto tile_body = [&](int32_t tile) -> bool {
    const int64_t s0 = sb + (int64_t)tile * 64;
    if (s0 >= se) return false;  // uniform over a heavy block
    const int lane = threadIdx.x & 63;
    const int64_t s = s0 + lane;
    const bool seg_ok = s < se;
    const int64_t i0 = seg_ok ? seg_start[s] : en.first;
    const int64_t i1 = seg_ok ? (s + 1 < se ? (int64_t)seg_start[s + 1] : en.first + en.count) : en.first + 1;
    const int len = (int)(i1 - i0);  // 1 .. kRecLen
    const CrystalPlan &P = plan[it.crystal];
    const double h = hh[i0], k = kk[i0], l0 = ll[i0];
    double s2d[R], lpv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = i0 + min(u, len - 1);
      s2d[u] = 0.25 * qq[i];
      lpv[u] = lpp[i];
    }
    // q(l0 + 1) - q(l0) from the metric (exact for the row, also past its end)
    const double dq0 = P.gs[2] * (2.0 * l0 + 1.0) + 2.0 * (P.gs[4] * h + P.gs[5] * k);
    const int na = it.atom_end - it.atom_begin;
    const int qn = (na + ww.nparts - 1) / ww.nparts;
    const int wa = it.atom_begin + min(na, ww.part * qn), wb = it.atom_begin + min(na, (ww.part + 1) * qn);
    double acc[V][R];
    rec_sums<MIXED, DERIV>(runs + it.run_begin, run_count[it.crystal], wa, wb, atoms, rot, coeff, coeff_f, h, k, l0,
                           s2d, dq0, acc);
    if (ww.heavy) {
      auto at = [&](int v, int u) -> double & { return s_red[(v * R + u) * 64 + lane]; };
      for (int w = ww.nparts - 1; w >= 1; --w) {
        if (ww.part == w) {
#pragma unroll
          for (int v = 0; v < V; ++v)
#pragma unroll
            for (int u = 0; u < R; ++u) at(v, u) = w == ww.nparts - 1 ? acc[v][u] : at(v, u) + acc[v][u];
        }
        __syncthreads();
      }
      if (ww.part != 0) return false;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u = 0; u < R; ++u) acc[v][u] = at(v, u) + acc[v][u];
    }
    if (!seg_ok) return true;
    const int64_t r0 = refl_offset[it.crystal], r1 = refl_offset[it.crystal + 1];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (u >= len) break;
      const int64_t i = i0 + u;
      const double A = acc[0][u], B = acc[1][u];
      const double I = (A * A + B * B) * lpv[u];
      Iout[i] = I;
      if constexpr (DERIV) store_derivs<MIXED>(cache, i, A, B, acc[2][u], acc[3][u]);
      const int64_t m = r0 + r1 - 1 - i;
      if constexpr (MIXED) {
        float *Af = (float *)Aout;
        float *Bf = (float *)Bout;
        Af[i] = (float)A;
        Bf[i] = (float)B;
        if (FRIEDEL) {
          Af[m] = (float)A;
          Bf[m] = -(float)B;
          Iout[m] = I;
        }
      } else {
        double *Ad = (double *)Aout;
        double *Bd = (double *)Bout;
        Ad[i] = A;
        Bd[i] = B;
        if (FRIEDEL) {
          Ad[m] = A;
          Bd[m] = -B;
          Iout[m] = I;
        }
      }
    }
    return true;
  };
  for (int32_t tile = it.tile; tile_body(tile) && it.tail; ++tile) {
  }
}

template <bool MIXED, bool FRIEDEL, bool DERIV>
void launch_rec_t(dim3 grid, const SfRecArgs &a, void *A, void *B, double *I, void *cache, hipStream_t s) {
  hipLaunchKernelGGL((k_sf_rec<MIXED, FRIEDEL, DERIV>), grid, dim3(kThreads), 0, s, a.items, a.n_items, a.n_heavy,
                     a.plan, a.refl_offset, a.seg_index, a.seg_start, a.h, a.k, a.l, a.q, a.lp, a.atoms, a.rot,
                     a.runs, a.run_count, a.coeff, a.coeff_f, A, B, I, cache);
}

}  // namespace

void launch_sf_rec(bool mixed, bool friedel, const SfRecArgs &a, void *A, void *B, double *I, void *deriv_cache,
                   hipStream_t s) {
  if (a.n_c <= 0) return;
  // segments of the current reflections: counts, their scan, starts
  if (a.n_eblocks > 0) {
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)a.n_eblocks), dim3(kThreads), 0, s, a.eblocks, a.n_c,
                       a.refl_offset, friedel, a.rec_of, a.h, a.k, a.l, a.seg_cnt, a.n_entries);
  } else {
    launch_fill_u64(reinterpret_cast<uint64_t *>(a.n_entries), 1, 0, s);
  }
  launch_scan_i32(a.seg_cnt, a.entry_cap, a.n_entries, const_cast<int64_t *>(a.seg_index), a.seg_part, s);
  if (a.n_eblocks > 0)
    hipLaunchKernelGGL(k_seg_write, dim3((unsigned)a.n_eblocks), dim3(kThreads), 0, s, a.eblocks, a.refl_offset,
                       friedel, a.seg_cnt, a.seg_index, const_cast<int32_t *>(a.seg_start));
  if (a.n_items <= 0) return;
  const dim3 grid((unsigned)(a.n_heavy + (a.n_items - a.n_heavy + 3) / 4));
  const bool d = deriv_cache != nullptr;
  if (mixed) {
    if (friedel)
      d ? launch_rec_t<true, true, true>(grid, a, A, B, I, deriv_cache, s)
        : launch_rec_t<true, true, false>(grid, a, A, B, I, deriv_cache, s);
    else
      d ? launch_rec_t<true, false, true>(grid, a, A, B, I, deriv_cache, s)
        : launch_rec_t<true, false, false>(grid, a, A, B, I, deriv_cache, s);
  } else {
    if (friedel)
      d ? launch_rec_t<false, true, true>(grid, a, A, B, I, deriv_cache, s)
        : launch_rec_t<false, true, false>(grid, a, A, B, I, deriv_cache, s);
    else
      d ? launch_rec_t<false, false, true>(grid, a, A, B, I, deriv_cache, s)
        : launch_rec_t<false, false, false>(grid, a, A, B, I, deriv_cache, s);
  }
}

}  // namespace xrd
