// Structure factors (paper, Section 2: the nested loops summing atomic
// contributions for each reflection, with the Debye-Waller and
// Lorentz-polarisation corrections; Section 4.2: this is where the time goes
// for large cells).
//
//   F(hkl) = sum_t f_t(s) sum_{j in t} occ_j exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j))
//
// Atoms are first packed per crystal and sorted by species (a stable
// partition), so the Cromer-Mann factor f_t(s) is evaluated once per
// (reflection, species) and multiplies a partial sum over that species'
// atoms instead of every term.
//
// One wavefront owns one work item: a tile of 64 x R reflections of one
// crystal (R, the reflections per lane, is the batch's tile shape: 1, 2 or 4).
// It walks the crystal's atoms in order; the atom index is uniform across the
// wavefront, so the atom records stream through the scalar cache into SGPRs
// and are broadcast to every lane with no LDS traffic and no barrier.  Each
// lane keeps R reflections in registers.
//
// Mixed precision (XRD_MIXED): t = h x + k y + l z in double, reduced mod 1
// in double (v_fract_f64), then sin/cos of the revolution in single precision
// by v_sin_f32 / v_cos_f32 (which take revolutions); weights
// occ exp(-B s^2) = exp2(log2(occ) - B log2(e) s^2) in single precision;
// single-precision sums over runs of at most kAtomTile atoms of one species,
// each multiplied by f_t and added in double (a product of two singles is
// exact in double, so the only single-precision roundings are inside a run).
// Plain path (XRD_FP64): the same loop in double with sincospi.
//
// Friedel: F(-h) = conj F(h) for real scattering factors, so with the option
// on only the positive half of each crystal's shell is evaluated and the
// conjugate is written to the mirror position.
#include <math.h>

#include <type_traits>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = kSfThreads;
constexpr int kAtomTile = 64;  // atoms per single-precision partial sum
constexpr double kLn2 = 0.69314718055994530942;

// ---- structure factors -----------------------------------------------------

// Sum over the 64 lanes of a wavefront with DPP row shifts and row
// broadcasts (VALU only); the total lands in lane 63.  Lanes a shift reads
// from outside their row contribute 0 (bound_ctrl); rows a broadcast does not
// write keep their value (old = 0 is added).
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xf, BOUND);
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(dpp_i32<CTRL, ROW_MASK, BOUND>(__float_as_int(x)));
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i32<CTRL, ROW_MASK, BOUND>((int)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL, ROW_MASK, BOUND>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float wave_sum_to_63(float v) {
  v += dpp_f32<0x111, 0xf, true>(v);   // row_shr:1
  v += dpp_f32<0x112, 0xf, true>(v);   // row_shr:2
  v += dpp_f32<0x114, 0xf, true>(v);   // row_shr:4
  v += dpp_f32<0x118, 0xf, true>(v);   // row_shr:8: lane 15 of each row holds the row sum
  v += dpp_f32<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f32<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ double wave_sum_to_63(double v) {
  v += dpp_f64<0x111, 0xf, true>(v);
  v += dpp_f64<0x112, 0xf, true>(v);
  v += dpp_f64<0x114, 0xf, true>(v);
  v += dpp_f64<0x118, 0xf, true>(v);
  v += dpp_f64<0x142, 0xa, false>(v);
  v += dpp_f64<0x143, 0xc, false>(v);
  return v;
}

// Six per-lane doubles summed over the wavefront at once by halving: at
// lane distances 32, 16 and 8 each lane keeps one value of every pair (the
// one its lane bit selects) plus its partner's copy of that value, then
// three exchanges finish the one value left.  Lane l ends with the wave
// total of value 4 ((l >> 3) & 1) + 2 ((l >> 4) & 1) + ((l >> 5) & 1)
// (values 6 and 7 are zero padding).
__device__ __forceinline__ double wave_reduce6(const double (&r)[6], int lane) {
  double v[8] = {r[0], r[1], r[2], r[3], r[4], r[5], 0.0, 0.0};
#pragma unroll
  for (int step = 0; step < 3; ++step) {
    const int m = 32 >> step, pairs = 4 >> step;
    const bool b = (lane & m) != 0;
    double nv[4];
#pragma unroll
    for (int i = 0; i < pairs; ++i) {
      const double send = b ? v[2 * i] : v[2 * i + 1];
      const double keep = b ? v[2 * i + 1] : v[2 * i];
      nv[i] = keep + __shfl_xor(send, m, 64);
    }
#pragma unroll
    for (int i = 0; i < pairs; ++i) v[i] = nv[i];
  }
  double x = v[0];
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  return x;
}

// Sixteen per-lane values reduced over the wavefront at once, with no
// selects for the two cross-row levels: v_permlane32_swap exchanges the upper
// half-wave of one register with the lower half of another, so pairing
// values (2i, 2i+1) and adding leaves value 2i + (lane >= 32) summed over
// lanes l and l ^ 32; v_permlane16_swap does the same with odd and even rows
// (pairs of those sums), leaving in row r value 4i + {0, 2, 1, 3}[r] summed
// over the four rows.  Within rows, a mirror and a half-mirror butterfly
// (each lane keeping the half whose index bit matches its lane bit 3, then
// bit 2) and two quad exchanges finish the sum.  On return lane l holds the
// wave total of value 4 ((l >> 2) & 3) + {0, 2, 1, 3}[l >> 4] (the same in
// the four lanes of its quad).
__device__ __forceinline__ int wave_reduce16_index(int lane) {
  const int rv = (lane >> 4) == 1 ? 2 : (lane >> 4) == 2 ? 1 : (lane >> 4);
  return 4 * ((lane >> 2) & 3) + rv;
}
__device__ __forceinline__ float wave_reduce16(const float (&v)[16], int lane) {
  float a[8], b[4], c[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i]), __float_as_uint(v[2 * i + 1]), false,
                                                    false);
    a[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[2 * i]), __float_as_uint(a[2 * i + 1]), false,
                                                    false);
    b[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int j = 0; j < 2; ++j) c[j] = (b3 ? b[2 + j] : b[j]) + dpp_f32<0x140, 0xf, false>(b3 ? b[j] : b[2 + j]);
  float w = (b2 ? c[1] : c[0]) + dpp_f32<0x141, 0xf, false>(b2 ? c[0] : c[1]);
  w += dpp_f32<0xb1, 0xf, false>(w);  // quad_perm [1, 0, 3, 2]
  w += dpp_f32<0x4e, 0xf, false>(w);  // quad_perm [2, 3, 0, 1]
  return w;
}

// Cromer-Mann factor at s^2 in single precision via exp2, from the
// species' single-precision table.
__device__ __forceinline__ float fsc_f32(const CoeffF &cf, float s2) {
  float f = cf.c;
#pragma unroll
  for (int i = 0; i < 4; ++i) f = fmaf(cf.a[i], __builtin_amdgcn_exp2f(cf.nbl[i] * s2), f);
  return f;
}

__device__ __forceinline__ double fsc_f64(const double *__restrict__ c9, double s2) {
  double f = c9[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) f = fma(c9[i], exp(-c9[4 + i] * s2), f);
  return f;
}

// Which part of the batch a wavefront takes.  Items (crystal, tile of 64 R
// evaluated reflections) come heavy first: the first n_heavy items get a block
// each, whose four wavefronts split the crystal's atoms into contiguous
// quarters (their sums are combined in LDS in wave order); the remaining
// items go four to a block, one per wavefront.  The wavefront index is made
// uniform so that everything derived from the item (crystal, runs, atom
// records) is loaded once per wave into SGPRs.
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

// Atom range [wa, wb) of a wavefront's part of the item's crystal.
__device__ __forceinline__ void part_range(const SfItem &it, const WaveWork &w, int *wa, int *wb) {
  const int na = it.atom_end - it.atom_begin;
  const int q = (na + w.nparts - 1) / w.nparts;
  *wa = it.atom_begin + min(na, w.part * q);
  *wb = it.atom_begin + min(na, (w.part + 1) * q);
}

// d f / d(s^2) alongside f (single and double precision); f takes the same
// operations as fsc_f32.
__device__ __forceinline__ void fsc_df_f32(const CoeffF &cf, float s2, float *f, float *df) {
  float a = cf.c, d = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float e = __builtin_amdgcn_exp2f(cf.nbl[i] * s2);
    a = fmaf(cf.a[i], e, a);
    d = fmaf(cf.nab[i], e, d);
  }
  *f = a;
  *df = d;
}

__device__ __forceinline__ void fsc_df_f64(const double *__restrict__ c9, double s2, double *f, double *df) {
  double a = c9[8], d = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double e = exp(-c9[4 + i] * s2);
    a = fma(c9[i], e, a);
    d = fma(-c9[i] * c9[4 + i], e, d);
  }
  *f = a;
  *df = d;
}

// One tile's reflections (R per lane) summed over a wavefront's atom range
// [wa, wb) of crystal runs cr[0, nr):
//   A + iB = sum_t f_t S_t,                 S_t  = sum_{j in t} occ_j e^{-B_j s^2} e^{i phi_j}
// and with DERIV also
//   d(A + iB)/ds^2 = sum_t (f'_t S_t + f_t S'_t),  S'_t = sum_{j in t} (-B_j) occ_j e^{-B_j s^2} e^{i phi_j}
// with f'_t = -sum_i a_i b_i e^{-b_i s^2} (t runs over species).  A and B take
// the same operations with or without DERIV, so keeping the derivatives does
// not change the structure factors.  Heavy items: the four wavefronts' sums
// meet in LDS (s_part) and are added in wave order; returns false for the
// waves that hold no totals afterwards (all but wave 0 unless all_waves).
template <bool MIXED, bool DERIV, int R>
__device__ __forceinline__ bool sf_tile_sums(const WaveWork &ww, int lane, const SpeciesRun *__restrict__ cr, int nr,
                                             int wa, int wb, const AtomRec *__restrict__ atoms,
                                             const double *__restrict__ coeff,
                                             const CoeffF *__restrict__ coeff_f, const double (&h)[R],
                                             const double (&k)[R], const double (&l)[R],
                                             const double (&s2d)[R], const float (&s2)[R],
                                             double *s_part, bool all_waves, double (&A)[R],
                                             double (&B)[R], double (&dA)[R], double (&dB)[R]) {
  if constexpr (MIXED) {
    // per reflection: A, B and, with DERIV, dA, dB in double; each chunk of
    // up to kAtomTile atoms of a run is summed in single precision and added
    // in double (the products of two singles are exact there).  The chunk
    // sums for dF/ds^2 carry B log2(e) w in place of -B w (no per-atom
    // conversion of B); the factor -ln 2 joins f when they are added.
    constexpr int V = DERIV ? 4 : 2;
    double acc[V][R];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int u = 0; u < R; ++u) acc[v][u] = 0.0;
    for (int ir = 0; ir < nr; ++ir) {
      const SpeciesRun run = cr[ir];
      const int rb = max(run.begin, wa), re = min(run.end, wb);
      if (rb >= re) continue;
      const CoeffF cf = coeff_f[run.species];
      double f[R], df[R], fq[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        float ff, dd = 0.f;
        if constexpr (DERIV)
          fsc_df_f32(cf, s2[u], &ff, &dd);
        else
          ff = fsc_f32(cf, s2[u]);
        f[u] = ff;
        df[u] = dd;
        fq[u] = -kLn2 * f[u];
      }
      for (int j0 = rb; j0 < re; j0 += kAtomTile) {
        const int j1 = min(j0 + kAtomTile, re);
        float pa[R], pb[R], qa[R], qb[R];
#pragma unroll
        for (int u = 0; u < R; ++u) pa[u] = pb[u] = qa[u] = qb[u] = 0.f;
        auto term = [&](const AtomRec &a) {
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const double t = fma(h[u], a.x, fma(k[u], a.y, l[u] * a.z));
            const float rho = (float)__builtin_amdgcn_fract(t);
            const float sn = __builtin_amdgcn_sinf(rho);
            const float cs = __builtin_amdgcn_cosf(rho);
            const float w = __builtin_amdgcn_exp2f(fmaf(-a.bl2e, s2[u], a.log2occ));
            pa[u] = fmaf(w, cs, pa[u]);
            pb[u] = fmaf(w, sn, pb[u]);
            if constexpr (DERIV) {
              const float bw = a.bl2e * w;
              qa[u] = fmaf(bw, cs, qa[u]);
              qb[u] = fmaf(bw, sn, qb[u]);
            }
          }
        };
        // four records per round: their scalar loads are issued together
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
          const AtomRec a0 = atoms[j], a1 = atoms[j + 1], a2 = atoms[j + 2], a3 = atoms[j + 3];
          term(a0);
          term(a1);
          term(a2);
          term(a3);
        }
        for (; j < j1; ++j) term(atoms[j]);
#pragma unroll
        for (int u = 0; u < R; ++u) {
          acc[0][u] = fma(f[u], (double)pa[u], acc[0][u]);
          acc[1][u] = fma(f[u], (double)pb[u], acc[1][u]);
          if constexpr (DERIV) {
            acc[2][u] = fma(df[u], (double)pa[u], fma(fq[u], (double)qa[u], acc[2][u]));
            acc[3][u] = fma(df[u], (double)pb[u], fma(fq[u], (double)qb[u], acc[3][u]));
          }
        }
      }
    }
    if (ww.heavy) {
      auto at = [&](int w, int v, int u) -> double & { return s_part[((w * V + v) * R + u) * 64 + lane]; };
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u = 0; u < R; ++u) at(ww.part, v, u) = acc[v][u];
      __syncthreads();
      if (!all_waves && ww.part != 0) return false;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u = 0; u < R; ++u) {
          acc[v][u] = at(0, v, u);
          for (int w = 1; w < kThreads / 64; ++w) acc[v][u] += at(w, v, u);
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      A[u] = acc[0][u];
      B[u] = acc[1][u];
      if constexpr (DERIV) {
        dA[u] = acc[2][u];
        dB[u] = acc[3][u];
      }
    }
  } else {
    constexpr int V = DERIV ? 4 : 2;
    double acc[V][R];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int u = 0; u < R; ++u) acc[v][u] = 0.0;
    for (int ir = 0; ir < nr; ++ir) {
      const SpeciesRun run = cr[ir];
      const int rb = max(run.begin, wa), re = min(run.end, wb);
      if (rb >= re) continue;
      const double *c9 = coeff + 9 * run.species;
      double f[R], df[R], pa[R], pb[R], qa[R], qb[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if constexpr (DERIV)
          fsc_df_f64(c9, s2d[u], &f[u], &df[u]);
        else
          f[u] = fsc_f64(c9, s2d[u]);
        pa[u] = pb[u] = qa[u] = qb[u] = 0.0;
      }
      for (int j = rb; j < re; ++j) {
        const AtomRec a = atoms[j];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const double t = fma(h[u], a.x, fma(k[u], a.y, l[u] * a.z));
          const double rho = t - rint(t);
          double sn, cs;
          sincospi(2.0 * rho, &sn, &cs);
          const double w = a.occ * exp(-a.bfac * s2d[u]);
          pa[u] = fma(w, cs, pa[u]);
          pb[u] = fma(w, sn, pb[u]);
          if constexpr (DERIV) {
            const double nbw = -a.bfac * w;
            qa[u] = fma(nbw, cs, qa[u]);
            qb[u] = fma(nbw, sn, qb[u]);
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
    if (ww.heavy) {
      auto at = [&](int w, int v, int u) -> double & { return s_part[((w * V + v) * R + u) * 64 + lane]; };
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u = 0; u < R; ++u) at(ww.part, v, u) = acc[v][u];
      __syncthreads();
      if (!all_waves && ww.part != 0) return false;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u = 0; u < R; ++u) {
          acc[v][u] = at(0, v, u);
          for (int w = 1; w < kThreads / 64; ++w) acc[v][u] += at(w, v, u);
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      A[u] = acc[0][u];
      B[u] = acc[1][u];
      if constexpr (DERIV) {
        dA[u] = acc[2][u];
        dB[u] = acc[3][u];
      }
    }
  }
  return true;
}

// Per-reflection values a later adjoint needs from the forward sums:
// (A, B, dA/ds^2, dB/ds^2), float4 under mixed precision, else double4,
// at the reflection's global index.
template <bool MIXED>
__device__ __forceinline__ void store_derivs(void *cache, int64_t i, double A, double B, double dA, double dB) {
  if constexpr (MIXED)
    reinterpret_cast<float4 *>(cache)[i] = make_float4((float)A, (float)B, (float)dA, (float)dB);
  else
    reinterpret_cast<double4 *>(cache)[i] = make_double4(A, B, dA, dB);
}

template <bool MIXED>
__device__ __forceinline__ void load_derivs(const void *cache, int64_t i, double *A, double *B, double *dA, double *dB) {
  if constexpr (MIXED) {
    const float4 v = reinterpret_cast<const float4 *>(cache)[i];
    *A = v.x;
    *B = v.y;
    *dA = v.z;
    *dB = v.w;
  } else {
    const double4 v = reinterpret_cast<const double4 *>(cache)[i];
    *A = v.x;
    *B = v.y;
    *dA = v.z;
    *dB = v.w;
  }
}

// Structure factors of one tile per wavefront (light items) or per block
// (heavy items).  With DERIV the derivatives with respect to s^2 are also
// summed and kept in ``cache`` for the adjoint.
template <bool MIXED, bool FRIEDEL, bool DERIV, int R>
__global__ __launch_bounds__(kThreads) void k_sf(const SfItem *__restrict__ items, int64_t n_items, int64_t n_heavy,
                                                 const int64_t *__restrict__ refl_offset,
                                                 const int16_t *__restrict__ hh, const int16_t *__restrict__ kk,
                                                 const int16_t *__restrict__ ll, const double *__restrict__ qq,
                                                 const double *__restrict__ lpp, const AtomRec *__restrict__ atoms,
                                                 const SpeciesRun *__restrict__ runs,
                                                 const int32_t *__restrict__ run_count,
                                                 const double *__restrict__ coeff,
                                                 const CoeffF *__restrict__ coeff_f, void *__restrict__ Aout,
                                                 void *__restrict__ Bout, double *__restrict__ Iout,
                                                 void *__restrict__ cache) {
  // heavy blocks: per wave, the doubles of each value (A, B and with DERIV
  // dA, dB), per reflection slot and lane
  __shared__ double s_part[(kThreads / 64) * (DERIV ? 4 : 2) * R * 64];
  const WaveWork ww = wave_work(n_heavy);
  if (ww.item >= n_items) return;  // light blocks only: a heavy block's item always exists
  const SfItem it = items[ww.item];
  const int64_t r0 = refl_offset[it.crystal], r1 = refl_offset[it.crystal + 1];
  const int64_t nref = r1 - r0;
  const int64_t first = FRIEDEL ? r0 + nref / 2 : r0;
  const int64_t count = FRIEDEL ? nref / 2 : nref;
  // a tail item walks the crystal's tiles from its first one on (the tiles
  // beyond the expected reflection count, which are mostly empty)
  auto tile_body = [&](int32_t tile) -> bool {
    const int64_t tbase = (int64_t)tile * (64 * R);
    if (tbase >= count) return false;  // uniform over a heavy block
    const int lane = threadIdx.x & 63;
    int64_t idx[R];
    bool valid[R];
    double h[R], k[R], l[R], s2d[R], lpv[R];
    float s2[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t t = tbase + u * 64 + lane;
      valid[u] = t < count;
      idx[u] = first + (valid[u] ? t : 0);
      h[u] = hh[idx[u]];
      k[u] = kk[idx[u]];
      l[u] = ll[idx[u]];
      s2d[u] = 0.25 * qq[idx[u]];
      s2[u] = (float)s2d[u];
      lpv[u] = lpp[idx[u]];  // loaded with the rest, not after the sums
    }
    int wa, wb;
    part_range(it, ww, &wa, &wb);
    double A[R], B[R], dA[R], dB[R];
    if (!sf_tile_sums<MIXED, DERIV, R>(ww, lane, runs + it.run_begin, run_count[it.crystal], wa, wb, atoms, coeff, coeff_f,
                                    h, k, l, s2d, s2, s_part, false, A, B, dA, dB))
      return false;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (!valid[u]) continue;
      const double I = (A[u] * A[u] + B[u] * B[u]) * lpv[u];
      Iout[idx[u]] = I;
      if constexpr (DERIV) store_derivs<MIXED>(cache, idx[u], A[u], B[u], dA[u], dB[u]);
      const int64_t m = r0 + r1 - 1 - idx[u];
      if constexpr (MIXED) {
        float *Af = (float *)Aout;
        float *Bf = (float *)Bout;
        Af[idx[u]] = (float)A[u];
        Bf[idx[u]] = (float)B[u];
        if (FRIEDEL) {
          Af[m] = (float)A[u];
          Bf[m] = -(float)B[u];
          Iout[m] = I;
        }
      } else {
        double *Ad = (double *)Aout;
        double *Bd = (double *)Bout;
        Ad[idx[u]] = A[u];
        Bd[idx[u]] = B[u];
        if (FRIEDEL) {
          Ad[m] = A[u];
          Bd[m] = -B[u];
          Iout[m] = I;
        }
      }
    }
    return true;
  };
  for (int32_t tile = it.tile; tile_body(tile) && it.tail; ++tile) {
  }
}


// ---- adjoint ---------------------------------------------------------------
//
// Reflection-major pass: for each evaluated reflection take A, B and their
// derivatives with respect to s^2 (kept by the forward, or summed again over
// the atoms); then, with gI = dL/dI summed over the reflection and (when
// Friedel pairing is on) its mate,
//   gA = 2 LP A gI,  gB = 2 LP B gI,
//   dL/dq = gI |F|^2 dLP/dq + (gA dA/ds^2 + gB dB/ds^2) / 4 + m w2 I d(2theta)/dq,
// where w1, w2 come from the grid adjoint and m = 2 with pairing, else 1.
template <bool MIXED, bool CACHED, int R>
__global__ __launch_bounds__(kThreads) void k_sf_bw(const SfItem *__restrict__ items, int64_t n_items, int64_t n_heavy, bool friedel,
                                                    const CrystalPlan *__restrict__ plan,
                                                    const int64_t *__restrict__ refl_offset,
                                                    const int16_t *__restrict__ hh, const int16_t *__restrict__ kk,
                                                    const int16_t *__restrict__ ll, const double *__restrict__ qq,
                                                    const double *__restrict__ lpp, double lambda,
                                                    const AtomRec *__restrict__ atoms,
                                                    const SpeciesRun *__restrict__ runs,
                                                    const int32_t *__restrict__ run_count,
                                                    const double *__restrict__ coeff,
                                                    const CoeffF *__restrict__ coeff_f, const void *__restrict__ cache,
                                                    const double2 *__restrict__ w12, double *__restrict__ ga,
                                                    double *__restrict__ gb, double *__restrict__ dq,
                                                    double *__restrict__ part6, double4 *__restrict__ part_fused) {
  // heavy blocks without the kept derivatives: per wave, value (8 floats or
  // 4 doubles), reflection slot, lane
  __shared__ double s_part[CACHED ? 1 : (kThreads / 64) * 4 * R * 64];
  const WaveWork ww = wave_work(n_heavy);
  if (ww.item >= n_items) return;  // light blocks only
  const SfItem it = items[ww.item];
  const int64_t r0 = refl_offset[it.crystal], r1 = refl_offset[it.crystal + 1];
  const int64_t nref = r1 - r0;
  const int64_t first = friedel ? r0 + nref / 2 : r0;
  const int64_t count = friedel ? nref / 2 : nref;
  // a tail item walks the crystal's tiles from its first one on
  auto tile_body = [&](int32_t tile) -> bool {
    const int64_t tbase = (int64_t)tile * (64 * R);
    if (tbase >= count) return false;
    const int lane = threadIdx.x & 63;
    int64_t idx[R];
    bool valid[R];
    double h[R], k[R], l[R], s2d[R];
    float s2[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t t = tbase + u * 64 + lane;
      valid[u] = t < count;
      idx[u] = first + (valid[u] ? t : 0);
      h[u] = hh[idx[u]];
      k[u] = kk[idx[u]];
      l[u] = ll[idx[u]];
      s2d[u] = 0.25 * qq[idx[u]];
      s2[u] = (float)s2d[u];
    }
    const CrystalPlan &P = plan[it.crystal];
    const SpeciesRun *cr = runs + it.run_begin;
    const int nr = run_count[it.crystal];
    int wa, wb;
    part_range(it, ww, &wa, &wb);
    double A[R], B[R], dA[R], dB[R];
    if constexpr (CACHED) {
#pragma unroll
      for (int u = 0; u < R; ++u) load_derivs<MIXED>(cache, idx[u], &A[u], &B[u], &dA[u], &dB[u]);
    } else {
      sf_tile_sums<MIXED, true, R>(ww, lane, cr, nr, wa, wb, atoms, coeff, coeff_f, h, k, l, s2d, s2, s_part, true, A, B,
                                dA, dB);
    }
    const double m = friedel ? 2.0 : 1.0;
    const double l2 = lambda * lambda;
    double gA[R], gB[R], dqv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      gA[u] = gB[u] = dqv[u] = 0.0;
      if (!valid[u]) continue;
      const int64_t i = idx[u];
      const double lp = lpp[i];
      const double2 wv = w12[i];
      const double gI = m * wv.x;
      gA[u] = 2.0 * lp * A[u] * gI;
      gB[u] = 2.0 * lp * B[u] * gI;
      // the other parts of a split item need gA and gB alone
      if (ww.part != 0) continue;
      const double q = qq[i];
      const double us = 0.25 * l2 * q;  // sin^2(theta)
      const double cs2 = 1.0 - us;      // cos^2(theta)
      const double sq = sqrt(cs2);
      // LP = num / den, num = 1 + (1 - 2 us)^2, den = us cos(theta); with
      // g = us cos^2(theta) and one reciprocal of it:
      //   dLP/dus = cos(theta) (2 cos^2 dnum us - num (2 - 3 us)) / (2 g^2),
      //   d(2theta)/dq = (180/pi) lambda^2 / (4 sqrt(g))  (= ... sqrt(g) / g)
      const double g = us * cs2, inv = 1.0 / g;
      const double num = 1.0 + (1.0 - 2.0 * us) * (1.0 - 2.0 * us);
      const double dnum = -4.0 * (1.0 - 2.0 * us);
      const double dlp_dq = sq * (2.0 * cs2 * dnum * us - num * (2.0 - 3.0 * us)) * (0.5 * inv * inv) * (0.25 * l2);
      const double dtt_dq = (180.0 / 3.14159265358979323846) * 0.25 * l2 * sqrt(g) * inv;
      const double f2 = A[u] * A[u] + B[u] * B[u];
      if (!P.fused) {
        ga[i] = gA[u];
        gb[i] = gB[u];
      }
      dqv[u] = gI * f2 * dlp_dq + 0.25 * (gA[u] * dA[u] + gB[u] * dB[u]) + m * wv.y * f2 * lp * dtt_dq;
      dq[i] = dqv[u];
    }
    if (ww.part == 0) {
      // the tile's row of dL/dG*: sum over its reflections of dL/dq times
      // (h^2, k^2, l^2, 2hk, 2hl, 2kl), as q = sum_ij G*_ij h_i h_j
      double r6[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) r6[e] = 0.0;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const double g = dqv[u];  // zero for lanes past the tile's end
        r6[0] += g * h[u] * h[u];
        r6[1] += g * k[u] * k[u];
        r6[2] += g * l[u] * l[u];
        r6[3] += 2.0 * g * h[u] * k[u];
        r6[4] += 2.0 * g * h[u] * l[u];
        r6[5] += 2.0 * g * k[u] * l[u];
      }
      const double tot = wave_reduce6(r6, lane);
      const int e6 = 4 * ((lane >> 3) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1);
      if ((lane & 7) == 0 && e6 < 6) part6[((int64_t)P.tile_begin + tile) * 6 + e6] = tot;
    }
    if (!P.fused) return true;
    // Fused atom gradients (small crystals): walk the atoms again; for each atom
    // the lanes' contributions from this tile's reflections are summed across
    // the wavefront and written as one partial row (tile, atom):
    //   (sum h P, sum k P, sum l P, sum s^2 Q),  P = w (gB cos - gA sin),
    //   Q = w (gA cos + gB sin),  w = occ f e^{-B s^2}.
    double4 *out = part_fused + P.pf_begin + (int64_t)tile * (P.atom_end - P.atom_begin);
    if constexpr (MIXED) {
      float hf[R], kf[R], lf[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        hf[u] = (float)h[u];
        kf[u] = (float)k[u];
        lf[u] = (float)l[u];
      }
      // four atoms per round over the wavefront's whole range, across species
      // runs: each atom takes the factors gA f_t, gB f_t of its run, formed
      // when the walk enters the run.  The records load together and the 16
      // sums (atom q, component c at index 4q + c) are reduced in one
      // butterfly; lane 4q + c then writes component c of atom q (records
      // past the range's end are re-read copies of its last atom and are not
      // written)
      int ir = 0, run_end = INT32_MIN;
      float fA[R], fB[R];
      for (int j0 = wa; j0 < wb; j0 += 4) {
        AtomRec a4[4];
        float fAq[4][R], fBq[4][R];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = min(j0 + q, wb - 1);
          a4[q] = atoms[j];
          if (j >= run_end) {
            while (cr[ir].end <= j) ++ir;
            const SpeciesRun run = cr[ir];
            run_end = run.end;
            const CoeffF cf = coeff_f[run.species];
#pragma unroll
            for (int u = 0; u < R; ++u) {
              const float f = fsc_f32(cf, s2[u]);
              fA[u] = (float)gA[u] * f;
              fB[u] = (float)gB[u] * f;
            }
          }
#pragma unroll
          for (int u = 0; u < R; ++u) {
            fAq[q][u] = fA[u];
            fBq[q][u] = fB[u];
          }
        }
        float v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const AtomRec &a = a4[q];
          float sx = 0.f, sy = 0.f, sz = 0.f, sb = 0.f;
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const double t = fma(h[u], a.x, fma(k[u], a.y, l[u] * a.z));
            const float rho = (float)__builtin_amdgcn_fract(t);
            const float sn = __builtin_amdgcn_sinf(rho);
            const float cs = __builtin_amdgcn_cosf(rho);
            const float w = __builtin_amdgcn_exp2f(fmaf(-a.bl2e, s2[u], a.log2occ));
            const float pP = w * (fBq[q][u] * cs - fAq[q][u] * sn);
            const float pQ = w * (fAq[q][u] * cs + fBq[q][u] * sn);
            sx = fmaf(hf[u], pP, sx);
            sy = fmaf(kf[u], pP, sy);
            sz = fmaf(lf[u], pP, sz);
            sb = fmaf(s2[u], pQ, sb);
          }
          v[4 * q + 0] = sx;
          v[4 * q + 1] = sy;
          v[4 * q + 2] = sz;
          v[4 * q + 3] = sb;
        }
        const float tot = wave_reduce16(v, lane);
        const int vi = wave_reduce16_index(lane), q = vi >> 2;
        if ((lane & 3) == 0 && j0 + q < wb)
          reinterpret_cast<double *>(out + (j0 + q - P.atom_begin))[vi & 3] = (double)tot;
      }
      return true;
    }
    // plain path: one atom at a time per species run, f_t in double
    for (int ir = 0; ir < nr; ++ir) {
      const SpeciesRun run = cr[ir];
      if (max(run.begin, wa) >= min(run.end, wb)) continue;
      const double *c9 = coeff + 9 * run.species;
      double f[R], fA[R], fB[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        f[u] = fsc_f64(c9, s2d[u]);
        fA[u] = gA[u] * f[u];
        fB[u] = gB[u] * f[u];
      }
      for (int j = max(run.begin, wa); j < min(run.end, wb); ++j) {
        const AtomRec a = atoms[j];
        double sx = 0.0, sy = 0.0, sz = 0.0, sb = 0.0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const double t = fma(h[u], a.x, fma(k[u], a.y, l[u] * a.z));
          const double rho = t - rint(t);
          double sn, cs;
          sincospi(2.0 * rho, &sn, &cs);
          const double w = a.occ * exp(-a.bfac * s2d[u]);
          const double pP = w * (fB[u] * cs - fA[u] * sn);
          const double pQ = w * (fA[u] * cs + fB[u] * sn);
          sx = fma(h[u], pP, sx);
          sy = fma(k[u], pP, sy);
          sz = fma(l[u], pP, sz);
          sb = fma(s2d[u], pQ, sb);
        }
        sx = wave_sum_to_63(sx);
        sy = wave_sum_to_63(sy);
        sz = wave_sum_to_63(sz);
        sb = wave_sum_to_63(sb);
        if (lane == 63) out[j - P.atom_begin] = make_double4(sx, sy, sz, sb);
      }
    }
    return true;
  };
  for (int32_t tile = it.tile; tile_body(tile) && it.tail; ++tile) {
  }
}

// Atom-major pass: block = (crystal, up to 256 atoms, chunk of kHalfChunk
// evaluated reflections).  Reflection tiles are staged in LDS with the
// scattering factor of every species of the crystal; each thread accumulates
// for its atom
//   dx += h P, dy += k P, dz += l P with P = w (gB cos phi - gA sin phi),
//   dB += s^2 Q with Q = w (gA cos phi + gB sin phi),   w = occ f e^{-B s^2}.
// A block whose crystal has A < 256 atoms splits into S = 256 / A slices that
// take every S-th reflection of a tile; the slices' sums are added in slice
// order through LDS, so the result does not depend on scheduling.  Writes the
// chunk's partial sums (the reduction applies 2 pi and the sign of dB).
template <bool MIXED>
__global__ __launch_bounds__(kThreads) void k_atom_bw(const BwItem *__restrict__ items, bool friedel,
                                                      const CrystalPlan *__restrict__ plan,
                                                      const int64_t *__restrict__ refl_offset,
                                                      const int16_t *__restrict__ hh, const int16_t *__restrict__ kk,
                                                      const int16_t *__restrict__ ll, const double *__restrict__ qq,
                                                      const double *__restrict__ ga, const double *__restrict__ gb,
                                                      const AtomRec *__restrict__ atoms,
                                                      const SpeciesRun *__restrict__ runs,
                                                      const int32_t *__restrict__ run_count,
                                                      const double *__restrict__ coeff,
                                                      const CoeffF *__restrict__ coeff_f, int tile, int runs_cap,
                                                      double4 *__restrict__ part) {
  using real = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  double *th = (double *)smem;
  double *tk = th + tile;
  double *tl = tk + tile;
  real *ts2 = (real *)(tl + tile);
  real *tga = ts2 + tile;
  real *tgb = tga + tile;
  real *tf = tgb + tile;           // [tile][runs_cap]
  // [runs_cap][9]: the crystal's species coefficients, (a_i, b_i, c) in
  // double, (a_i, -b_i log2(e), c) from the single-precision table
  real *tcoef = tf + tile * runs_cap;

  const BwItem it = items[blockIdx.x];
  const CrystalPlan &P = plan[it.crystal];
  const int64_t r0 = refl_offset[it.crystal], r1 = refl_offset[it.crystal + 1];
  const int64_t nref = r1 - r0;
  const int64_t first = friedel ? r0 + nref / 2 : r0;
  const int64_t count = friedel ? nref / 2 : nref;
  const int64_t na = P.atom_end - P.atom_begin;
  const int64_t a_base = (int64_t)it.ablock * kAtomBlock;
  const int A = (int)min((int64_t)kAtomBlock, na - a_base);  // atoms of this block (>= 1)
  const int S = kThreads / A;                                // slices
  const int slice = threadIdx.x / A, al = threadIdx.x - slice * A;
  const bool valid = slice < S;
  const int64_t ja = a_base + (valid ? al : 0);  // atom within the crystal
  const int64_t j = P.atom_begin + ja;
  double4 *out = part + P.part_begin + (int64_t)it.chunk * na;
  const int64_t e0 = (int64_t)it.chunk * kHalfChunk;
  const int64_t e1 = min(e0 + (int64_t)kHalfChunk, count);
  if (e0 >= e1) {  // chunk beyond this crystal's reflections: zero partials
    if (valid && slice == 0) out[ja] = make_double4(0.0, 0.0, 0.0, 0.0);
    return;
  }
  const SpeciesRun *cr = runs + P.run_begin;
  const int nr = run_count[it.crystal];
  int myrun = 0;
  for (int ir = 0; ir < nr; ++ir)
    if (j >= cr[ir].begin && j < cr[ir].end) myrun = ir;
  for (int x = threadIdx.x; x < nr * 9; x += kThreads) {
    const int ir = x / 9, q9 = x - ir * 9;
    if constexpr (MIXED) {
      const CoeffF &cf = coeff_f[cr[ir].species];
      tcoef[ir * 9 + q9] = q9 < 4 ? cf.a[q9] : q9 < 8 ? cf.nbl[q9 - 4] : cf.c;
    } else {
      tcoef[ir * 9 + q9] = coeff[9 * cr[ir].species + q9];
    }
  }
  const AtomRec a = atoms[j];
  double sx = 0.0, sy = 0.0, sz = 0.0, sB = 0.0;
  for (int64_t t0 = e0; t0 < e1; t0 += tile) {
    __syncthreads();
    for (int r = threadIdx.x; r < tile; r += kThreads) {
      const int64_t e = t0 + r;
      if (e < e1) {
        const int64_t i = first + e;
        th[r] = hh[i];
        tk[r] = kk[i];
        tl[r] = ll[i];
        ts2[r] = (real)(0.25 * qq[i]);
        tga[r] = (real)ga[i];
        tgb[r] = (real)gb[i];
      } else {
        th[r] = tk[r] = tl[r] = 0.0;
        ts2[r] = tga[r] = tgb[r] = (real)0;
      }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < tile * nr; x += kThreads) {
      const int r = x / nr, ir = x - r * nr;
      const real *c9 = tcoef + 9 * ir;
      real f = c9[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (MIXED) f = fmaf(c9[i], __builtin_amdgcn_exp2f(c9[4 + i] * ts2[r]), f);
        else f = fma(c9[i], exp(-c9[4 + i] * ts2[r]), f);
      }
      tf[r * runs_cap + ir] = f;
    }
    __syncthreads();
    if (valid) {
      const int nt = (int)min((int64_t)tile, e1 - t0);
      real px = 0, py = 0, pz = 0, pB = 0;
      for (int r = slice; r < nt; r += S) {
        const double t = fma(th[r], a.x, fma(tk[r], a.y, tl[r] * a.z));
        real sn, cs, w;
        if constexpr (MIXED) {
          const float rho = (float)__builtin_amdgcn_fract(t);
          sn = __builtin_amdgcn_sinf(rho);
          cs = __builtin_amdgcn_cosf(rho);
          w = tf[r * runs_cap + myrun] * __builtin_amdgcn_exp2f(fmaf(-a.bl2e, ts2[r], a.log2occ));
        } else {
          const double rho = t - rint(t);
          sincospi(2.0 * rho, &sn, &cs);
          w = tf[r * runs_cap + myrun] * a.occ * exp(-a.bfac * ts2[r]);
        }
        const real pP = w * (tgb[r] * cs - tga[r] * sn);
        const real pQ = w * (tga[r] * cs + tgb[r] * sn);
        px += (real)th[r] * pP;
        py += (real)tk[r] * pP;
        pz += (real)tl[r] * pP;
        pB += ts2[r] * pQ;
      }
      sx += (double)px;
      sy += (double)py;
      sz += (double)pz;
      sB += (double)pB;
    }
  }
  // slice sums in slice order
  __syncthreads();
  double4 *red = (double4 *)smem;  // kThreads entries; the tile arrays are no longer needed
  red[threadIdx.x] = make_double4(sx, sy, sz, sB);
  __syncthreads();
  if (valid && slice == 0) {
    double4 v = red[al];
    for (int s2 = 1; s2 < S; ++s2) {
      const double4 o = red[s2 * A + al];
      v.x += o.x;
      v.y += o.y;
      v.z += o.z;
      v.w += o.w;
    }
    out[ja] = v;
  }
}

// Sum of the partials of each atom in a fixed order (tile order for fused
// crystals, chunk order otherwise); scatter to the caller's atom order.
// Sum of rows p[0], p[stride], ... p[(n - 1) stride] in row order, eight
// loads in flight at a time.
__device__ __forceinline__ void sum_rows(const double4 *__restrict__ p, int64_t stride, int64_t n, double *sx,
                                         double *sy, double *sz, double *sB) {
  double ax = 0.0, ay = 0.0, az = 0.0, ab = 0.0;
  int64_t t = 0;
  for (; t + 8 <= n; t += 8) {
    double4 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[(t + i) * stride];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ax += v[i].x;
      ay += v[i].y;
      az += v[i].z;
      ab += v[i].w;
    }
  }
  for (; t < n; ++t) {
    const double4 v = p[t * stride];
    ax += v.x;
    ay += v.y;
    az += v.z;
    ab += v.w;
  }
  *sx = ax;
  *sy = ay;
  *sz = az;
  *sB = ab;
}

__device__ __forceinline__ void atom_bw_reduce(const AbItem it, bool friedel, const CrystalPlan *__restrict__ plan,
                                               const int64_t *__restrict__ refl_offset,
                                               const double4 *__restrict__ part,
                                               const double4 *__restrict__ part_fused,
                                               const int32_t *__restrict__ orig, double *__restrict__ dfrac,
                                               double *__restrict__ dbfac) {
  const CrystalPlan &P = plan[it.crystal];
  const int64_t na = P.atom_end - P.atom_begin;
  const int64_t ja = (int64_t)it.ablock * kAtomBlock + threadIdx.x;
  if (ja >= na) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, sB = 0.0;
  if (P.fused) {
    const int64_t nref = refl_offset[it.crystal + 1] - refl_offset[it.crystal];
    const int64_t count = friedel ? nref / 2 : nref;
    const int64_t tiles = (count + P.sf_tile - 1) / P.sf_tile;  // tiles that ran
    const double4 *p = part_fused + P.pf_begin + ja;
    sum_rows(p, na, tiles, &sx, &sy, &sz, &sB);
  } else {
    const double4 *p = part + P.part_begin + ja;
    sum_rows(p, na, P.n_hchunks, &sx, &sy, &sz, &sB);
  }
  const double tp = 2.0 * 3.14159265358979323846;
  const int64_t o = orig[P.atom_begin + ja];
  dfrac[3 * o] = tp * sx;
  dfrac[3 * o + 1] = tp * sy;
  dfrac[3 * o + 2] = tp * sz;
  dbfac[o] = -sB;
}

// dL/dG* (its 6 unique entries, U) ->
// dL/d(a, b, c, alpha, beta, gamma), angles in degrees.  q = sum_ij M_ij h_i h_j
// with M = G*, so dL/dM_ij = U_ij for i == j and U_ij / 2 for i != j (the
// unique entry appears twice); dL/dG = -M (dL/dM) M.
__device__ void lattice_chain(const CrystalPlan &P, const double (&U)[6], double *__restrict__ o) {
  const double M[3][3] = {{P.gs[0], P.gs[3], P.gs[4]}, {P.gs[3], P.gs[1], P.gs[5]}, {P.gs[4], P.gs[5], P.gs[2]}};
  const double D[3][3] = {{U[0], 0.5 * U[3], 0.5 * U[4]}, {0.5 * U[3], U[1], 0.5 * U[5]}, {0.5 * U[4], 0.5 * U[5], U[2]}};
  double T[3][3], Gb[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += D[i][m] * M[m][j];
      T[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += M[i][m] * T[m][j];
      Gb[i][j] = -s;
    }
  const double a = P.lat[0], b = P.lat[1], cc = P.lat[2];
  const double rad = 3.14159265358979323846 / 180.0;
  double sa, ca, sb, cb, sg, cg;
  sincos(P.lat[3] * rad, &sa, &ca);
  sincos(P.lat[4] * rad, &sb, &cb);
  sincos(P.lat[5] * rad, &sg, &cg);
  // G11 = a^2, G22 = b^2, G33 = c^2, G12 = ab cos(gamma), G13 = ac cos(beta), G23 = bc cos(alpha);
  // off-diagonal entries appear twice in the full symmetric matrix.
  const double g12 = 2.0 * Gb[0][1], g13 = 2.0 * Gb[0][2], g23 = 2.0 * Gb[1][2];
  o[0] = Gb[0][0] * 2.0 * a + g12 * b * cg + g13 * cc * cb;
  o[1] = Gb[1][1] * 2.0 * b + g12 * a * cg + g23 * cc * ca;
  o[2] = Gb[2][2] * 2.0 * cc + g13 * a * cb + g23 * b * ca;
  o[3] = g23 * (-b * cc * sa * rad);
  o[4] = g13 * (-a * cc * sb * rad);
  o[5] = g12 * (-a * b * sg * rad);
}

// The last step of the adjoint, two independent parts in one launch: blocks
// [0, n_ab) reduce the atom gradients (one thread per atom, its partial rows
// in order), the rest take one crystal per wavefront through the lattice
// chain rule, summing the crystal's structure-factor tile rows of dL/dG*
// (the tiles that ran).
__global__ __launch_bounds__(kThreads) void k_bw_finish(const AbItem *__restrict__ items, int64_t n_ab, bool friedel,
                                                        const CrystalPlan *__restrict__ plan, int64_t n_c,
                                                        const int64_t *__restrict__ refl_offset,
                                                        const double4 *__restrict__ part,
                                                        const double4 *__restrict__ part_fused,
                                                        const int32_t *__restrict__ orig,
                                                        const double *__restrict__ part6, double *__restrict__ dfrac,
                                                        double *__restrict__ dbfac, double *__restrict__ dlat) {
  if (blockIdx.x < n_ab) {
    atom_bw_reduce(items[blockIdx.x], friedel, plan, refl_offset, part, part_fused, orig, dfrac, dbfac);
    return;
  }
  // one wavefront per crystal: lane i sums rows i, i + 64, ... in order, the
  // wavefront adds the lanes' sums in a fixed pattern, lane 63 applies the
  // chain rule
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)(blockIdx.x - n_ab) * (kThreads / 64) + (threadIdx.x >> 6);
  if (c >= n_c) return;
  const CrystalPlan &P = plan[c];
  const int64_t nref = refl_offset[c + 1] - refl_offset[c];
  const int64_t count = friedel ? nref / 2 : nref;
  const int n_rows = (int)((count + P.sf_tile - 1) / P.sf_tile);
  const double *rows = part6 + (int64_t)P.tile_begin * 6;
  double U[6] = {0, 0, 0, 0, 0, 0};
  for (int k = lane; k < n_rows; k += 64)
#pragma unroll
    for (int e = 0; e < 6; ++e) U[e] += rows[k * 6 + e];
#pragma unroll
  for (int e = 0; e < 6; ++e) U[e] = wave_sum_to_63(U[e]);
  if (lane == 63) lattice_chain(P, U, dlat + 6 * c);
}

}  // namespace



template <bool MIXED, bool FRIEDEL, bool DERIV, int R>
static void launch_sf_t(dim3 grid, const SfItem *items, int64_t n_items, int64_t n_heavy,
                        const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l,
                        const double *q, const double *lp, const AtomRec *atoms, const SpeciesRun *runs,
                        const int32_t *run_count, const double *coeff, const CoeffF *coeff_f, void *A, void *B,
                        double *I, void *cache, hipStream_t s) {
  hipLaunchKernelGGL((k_sf<MIXED, FRIEDEL, DERIV, R>), grid, dim3(kThreads), 0, s, items, n_items, n_heavy,
                     refl_offset, h, k, l, q, lp, atoms, runs, run_count, coeff, coeff_f, A, B, I, cache);
}

void launch_sf(bool mixed, bool friedel, const SfItem *items, int64_t n_items, int64_t n_heavy, const CrystalPlan *plan,
               const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l, const double *q,
               const double *lp, const AtomRec *atoms, const SpeciesRun *runs, const int32_t *run_count,
               const double *coeff, const CoeffF *coeff_f, void *A, void *B, double *I, void *deriv_cache,
               int rpt, hipStream_t s) {
  if (n_items <= 0) return;
  const dim3 grid((unsigned)(n_heavy + (n_items - n_heavy + 3) / 4));
  auto go = [&](auto fn) {
    fn(grid, items, n_items, n_heavy, refl_offset, h, k, l, q, lp, atoms, runs, run_count, coeff, coeff_f, A, B,
       I, deriv_cache, s);
  };
  const bool d = deriv_cache != nullptr;
  // the instantiation for (precision, Friedel pairing, kept derivatives, R)
  auto by_r = [&](auto f1, auto f2, auto f4) { rpt == 1 ? go(f1) : rpt == 4 ? go(f4) : go(f2); };
#define XRD_SF_R(M, F, D) by_r(launch_sf_t<M, F, D, 1>, launch_sf_t<M, F, D, 2>, launch_sf_t<M, F, D, 4>)
  if (mixed) {
    if (friedel)
      d ? XRD_SF_R(true, true, true) : XRD_SF_R(true, true, false);
    else
      d ? XRD_SF_R(true, false, true) : XRD_SF_R(true, false, false);
  } else {
    if (friedel)
      d ? XRD_SF_R(false, true, true) : XRD_SF_R(false, true, false);
    else
      d ? XRD_SF_R(false, false, true) : XRD_SF_R(false, false, false);
  }
#undef XRD_SF_R
}

}  // namespace xrd

namespace xrd {

void launch_sf_bw(bool mixed, bool friedel, const SfItem *items, int64_t n_items, int64_t n_heavy,
                  const CrystalPlan *plan,
                  const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l, const double *q,
                  const double *lp, double lambda, const AtomRec *atoms, const SpeciesRun *runs,
                  const int32_t *run_count, const double *coeff, const CoeffF *coeff_f, const void *deriv_cache,
                  const double2 *w12, double *ga, double *gb, double *dq, double *part6, double *part_fused,
                  int rpt, hipStream_t s) {
  if (n_items <= 0) return;
  const dim3 grid((unsigned)(n_heavy + (n_items - n_heavy + 3) / 4)), block(kThreads);
  double4 *pf = (double4 *)part_fused;
#define XRD_SF_BW(M, C, R)                                                                                          \
  hipLaunchKernelGGL((k_sf_bw<M, C, R>), grid, block, 0, s, items, n_items, n_heavy, friedel, plan, refl_offset, h, \
                     k, l, q, lp, lambda, atoms, runs, run_count, coeff, coeff_f, deriv_cache, w12, ga, gb, dq,       \
                     part6, pf)
#define XRD_SF_BW_R(M, C)   \
  if (rpt == 1)             \
    XRD_SF_BW(M, C, 1);     \
  else if (rpt == 4)        \
    XRD_SF_BW(M, C, 4);     \
  else                      \
    XRD_SF_BW(M, C, 2)
  if (mixed) {
    if (deriv_cache) {
      XRD_SF_BW_R(true, true);
    } else {
      XRD_SF_BW_R(true, false);
    }
  } else {
    if (deriv_cache) {
      XRD_SF_BW_R(false, true);
    } else {
      XRD_SF_BW_R(false, false);
    }
  }
#undef XRD_SF_BW_R
#undef XRD_SF_BW
}

void launch_atom_bw(bool mixed, bool friedel, const BwItem *items, int64_t n_items, const CrystalPlan *plan,
                    const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l,
                    const double *q, const double *ga, const double *gb, const AtomRec *atoms,
                    const SpeciesRun *runs, const int32_t *run_count, const double *coeff, const CoeffF *coeff_f,
                    int tile, int runs_cap, double *part, hipStream_t s) {
  if (n_items <= 0) return;
  const size_t lds = atom_bw_lds_bytes(mixed, tile, runs_cap);
  const BwItem *it = items;
  if (mixed)
    hipLaunchKernelGGL(k_atom_bw<true>, dim3((unsigned)n_items), dim3(kThreads), lds, s, it, friedel, plan,
                       refl_offset, h, k, l, q, ga, gb, atoms, runs, run_count, coeff, coeff_f, tile, runs_cap,
                       (double4 *)part);
  else
    hipLaunchKernelGGL(k_atom_bw<false>, dim3((unsigned)n_items), dim3(kThreads), lds, s, it, friedel, plan,
                       refl_offset, h, k, l, q, ga, gb, atoms, runs, run_count, coeff, coeff_f, tile, runs_cap,
                       (double4 *)part);
}

void launch_bw_finish(const AbItem *items, int64_t n_ab, bool friedel, const CrystalPlan *plan, int64_t n_c,
                      const int64_t *refl_offset, const double *part, const double *part_fused, const int32_t *orig,
                      const double *part6, double *dfrac, double *dbfac, double *dlat, hipStream_t s) {
  const int64_t blocks = n_ab + (n_c + kThreads / 64 - 1) / (kThreads / 64);
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_bw_finish, dim3((unsigned)blocks), dim3(kThreads), 0, s, items, n_ab, friedel, plan, n_c,
                     refl_offset, (const double4 *)part, (const double4 *)part_fused, orig, part6, dfrac, dbfac,
                     dlat);
}


}  // namespace xrd
