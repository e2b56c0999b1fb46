// Gaussian broadening of the reflections onto a 2theta grid, and the grid side
// of its adjoint.  The paper motivates fast simulation with machine-learning
// datasets of patterns modified by peak broadening (Section 1); this is the
// differentiable pattern those models consume.
//
//   y_g = sum_r I_r K(x_g - 2theta_r),  K(d) = exp(-d^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
//   restricted to |x_g - 2theta_r| <= window * sigma, x_g = t0 + g dt.
//
// Both directions work on the entries that the sort leaves behind: each
// crystal's evaluated reflections in ascending 2theta.  Forward: a gather in
// which each lane owns one grid point and sums, in 2theta order, the entries
// whose window holds it, so the result is deterministic without atomics; a
// preparation pass gives every wave the entry range of its 64 points.
// Adjoint: per entry, w1 = sum_g dL/dy_g K and w2 = sum_g dL/dy_g K
// (x_g - 2theta) / sigma^2 over the same window; on the uniform grid the
// Gaussian follows a two-term multiplicative recurrence
//   K(d + dt) = K(d) r(d),  r(d) = exp(-(2 d dt + dt^2) / (2 sigma^2)),
//   r(d + dt) = r(d) rho,   rho = exp(-dt^2 / sigma^2),
// so a whole window costs two exp and a few products per point.
#include <math.h>

#include <type_traits>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GridArgs {
  double t0, dt, inv_dt, sigma, half, norm, inv2s2;
  int64_t n;
};

// Grid points covered by a reflection at 2theta t: the interval of g in
// [0, n) with |x_g - t| <= half, x_g = t0 + g dt (an interval because x_g - t
// is monotone in g).  Empty when lo > hi.
__device__ __forceinline__ void window_of(const GridArgs &g, double t, int64_t *lo, int64_t *hi) {
#pragma clang fp contract(off)
  // grid indices are carried as doubles (exact integers here): the
  // estimates, clamped to [-2, n + 1] so that the settling steps stay few
  const double n = (double)g.n;
  double a = fmin(fmax(ceil((t - g.half - g.t0) * g.inv_dt), -2.0), n + 1.0);
  double b = fmin(fmax(floor((t + g.half - g.t0) * g.inv_dt), -2.0), n + 1.0);
  // the estimates (a product with the rounded reciprocal) are off by at most
  // one step either way; settle them with the exact test
  while (a > 0.0 && fabs(g.t0 + (a - 1.0) * g.dt - t) <= g.half) a -= 1.0;
  while (a <= b && fabs(g.t0 + a * g.dt - t) > g.half) a += 1.0;
  while (b + 1.0 < n && fabs(g.t0 + (b + 1.0) * g.dt - t) <= g.half) b += 1.0;
  while (b >= a && fabs(g.t0 + b * g.dt - t) > g.half) b -= 1.0;
  *lo = (int64_t)fmax(a, 0.0);
  *hi = (int64_t)fmin(b, n - 1.0);
}

constexpr int kSegPts = 1024;                  // grid points per gather block (4 per thread)
constexpr int kGTile = 1024;                   // entries per LDS tile of the gather
constexpr int kAdjSpan = 4096;                 // grid points of dL/dy an adjoint block stages in LDS
static_assert(kSegPts == 64 * kSpanPts, "a gather block covers 64 spans, a quarter wavefront each");

// Entries: the evaluated reflections of a crystal in ascending 2theta (both
// mates of a Friedel pair share 2theta and I exactly, so with pairing one
// entry of weight 2 I stands for both).  Entry e of crystal c sits at
// base(c) + e, base = r0/2 with pairing and r0 without.
struct EntryRange {
  int64_t base, count;
};
__device__ __forceinline__ EntryRange entry_range(const int64_t *__restrict__ refl_offset, int64_t c, bool friedel) {
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  EntryRange e;
  e.base = friedel ? r0 / 2 : r0;
  e.count = friedel ? (r1 - r0) / 2 : r1 - r0;
  return e;
}

// Window of an entry as int32, clamped to [0, n] x [-1, n-1] (empty: lo > hi).
__device__ __forceinline__ int2 window32(const GridArgs &g, double t) {
  int64_t lo, hi;
  window_of(g, t, &lo, &hi);
  return make_int2((int)min(lo, g.n), (int)max(hi, (int64_t)-1));
}

// A window one step wider on each side than window_of's, from the rounded
// quotients alone (no exact tests), clamped like window32.  Nondecreasing in
// t; the forward uses it only to choose which entries a span walks, and the
// lanes' own |x - t| <= half test decides each point.
__device__ __forceinline__ int2 window_wide(const GridArgs &g, double t) {
  const double u = (t - g.t0) * g.inv_dt, hw = g.half * g.inv_dt, n = (double)g.n;
  const double lo = fmin(fmax(floor(u - hw) - 1.0, 0.0), n);
  const double hi = fmin(fmax(ceil(u + hw) + 1.0, -1.0), n - 1.0);
  return make_int2((int)lo, (int)hi);
}

// Entry preparation, one block per kEntBlock entries of a crystal: the
// weight w_e = m I norm of every entry, and the entry ranges of the
// crystal's spans of kSpanPts grid points:
//   first[s] = min{e : gh_e >= P s},  last[s] = max{e : gl_e <= P s + P - 1},
// P = kSpanPts, with [gl_e, gh_e] the (clamped, one step wide) window of
// entry e.  Both ends are nondecreasing in e, so entry e owns first[s] for s
// in (gh_{e-1} / P, gh_e / P] and last[s] for s in [gl_e / P, gl_{e+1} / P)
// (integer floors), the first and last entries also own the spans beyond;
// every span of a crystal with entries is written exactly once.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_entry_prep(const HChunk *__restrict__ eblocks,
                                                    const CrystalPlan *__restrict__ plan, bool friedel,
                                                    const int64_t *__restrict__ refl_offset,
                                                    const double *__restrict__ ent_key,
                                                    const int32_t *__restrict__ ent_idx,
                                                    const double *__restrict__ inten, GridArgs g, int64_t span_cap,
                                                    double *__restrict__ ent_w, int32_t *__restrict__ span_first,
                                                    int32_t *__restrict__ span_last) {
#pragma clang fp contract(off)
  __shared__ int32_t s_gl[kEntBlock + 2], s_gh[kEntBlock + 2];
  const HChunk hk = eblocks[blockIdx.x];
  const int32_t c = hk.crystal;
  const EntryRange er = entry_range(refl_offset, c, friedel);
  const int64_t e0 = (int64_t)hk.chunk * kEntBlock;
  if (e0 >= er.count) return;
  const int64_t e1 = min(e0 + (int64_t)kEntBlock, er.count);
  const int S = (int)((g.n + kSpanPts - 1) / kSpanPts);
  constexpr int U = kEntBlock / 256;
  // loads first, all at once: keys (and the two neighbours at the block's
  // ends), reflection indices, then intensities
  double key[U];
  int32_t idx[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t e = e0 + u * 256 + threadIdx.x;
    key[u] = e < e1 ? ent_key[er.base + e] : 0.0;
    idx[u] = e < e1 ? ent_idx[er.base + e] : 0;
  }
  double halo = 0.0;
  const int64_t eh = threadIdx.x == 0 ? e0 - 1 : e1;  // thread 0: left neighbour, thread 1: right
  const bool has_halo = threadIdx.x < 2 && eh >= 0 && eh < er.count;
  if (has_halo) halo = ent_key[er.base + eh];
  double iv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) iv[u] = e0 + u * 256 + threadIdx.x < e1 ? inten[idx[u]] : 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t e = e0 + u * 256 + threadIdx.x;
    if (e < e1) {
      const int2 w = window_wide(g, key[u]);
      s_gl[e - e0 + 1] = w.x;
      s_gh[e - e0 + 1] = w.y;
    }
  }
  if (has_halo) {
    const int2 w = window_wide(g, halo);
    s_gl[eh - e0 + 1] = w.x;
    s_gh[eh - e0 + 1] = w.y;
  }
  __syncthreads();
  const double m = friedel ? 2.0 : 1.0;
  int32_t *__restrict__ first = span_first + (int64_t)c * span_cap;
  int32_t *__restrict__ last = span_last + (int64_t)c * span_cap;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t e = e0 + u * 256 + threadIdx.x;
    if (e >= e1) continue;
    if constexpr (MIXED)
      reinterpret_cast<float *>(ent_w)[er.base + e] = (float)(m * iv[u] * g.norm);
    else
      ent_w[er.base + e] = m * iv[u] * g.norm;
    const int i = (int)(e - e0) + 1;
    const int gh = s_gh[i], gl = s_gl[i];
    const int fb = gh >= 0 ? gh / kSpanPts : -1;
    const int fa = e == 0 ? 0 : (s_gh[i - 1] >= 0 ? s_gh[i - 1] / kSpanPts : -1) + 1;
    for (int s = max(fa, 0); s <= min(fb, S - 1); ++s) first[s] = (int32_t)e;
    if (e == er.count - 1)
      for (int s = max(fb + 1, 0); s < S; ++s) first[s] = (int32_t)er.count;
    const int la = gl / kSpanPts;
    const int lb = e == er.count - 1 ? S - 1 : s_gl[i + 1] / kSpanPts - 1;
    for (int s = la; s <= min(lb, S - 1); ++s) last[s] = (int32_t)e;
    if (e == 0)
      for (int s = 0; s < min(la, S); ++s) last[s] = -1;
  }
}

// Forward gather: a block owns kSegPts consecutive grid points of one
// crystal, each lane four of them, 256 apart; for its j-th point, the
// sixteen lanes of quarter q of wave w cover span 16j + 4w + q of the
// segment.  The entries reaching the segment (first of its first span ..
// last of its last span) are staged in LDS in tiles; each quarter walks its
// span's entry range in 2theta order (a quarter's lanes read the same LDS
// entry; the wave runs as long as its longest range), and each lane adds
// w K(x - 2theta) when its point lies in the entry's window (the same
// |x - 2theta| <= half test that defines the window), so every point sums
// exactly its reflections, in sorted order, deterministically.  Spans of a
// quarter wavefront keep the share of entries that miss a lane's window
// small (a span of P points walks the entries of P points plus a window).  The offset
// x - 2theta and the window test are double precision in both paths; under
// MIXED the weight, the exponential (v_exp_f32) and the sums are single
// precision, otherwise double.  Blocks take the crystals heaviest first and
// each crystal's segments from the high-angle end, where reflections are
// densest, so the longest blocks start first.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_broaden_gather(const int32_t *__restrict__ crystal_order,
                                                        const int64_t *__restrict__ refl_offset, bool friedel,
                                                        const double *__restrict__ ent_key,
                                                        const double *__restrict__ ent_w,
                                                        const int32_t *__restrict__ span_first,
                                                        const int32_t *__restrict__ span_last, int64_t span_cap,
                                                        GridArgs g, double *__restrict__ y) {
#pragma clang fp contract(off)
  using real = typename std::conditional<MIXED, float, double>::type;
  // an entry is 16 bytes (2theta, weight, padding under MIXED), read with one
  // 128-bit LDS access
  __shared__ double2 s_ent[kGTile];
  const int S = (int)((g.n + kSpanPts - 1) / kSpanPts);
  const int segs = (int)((g.n + kSegPts - 1) / kSegPts);
  const int64_t c = crystal_order[blockIdx.x / segs];
  const int sb = (segs - 1 - (int)(blockIdx.x % segs)) * (kSegPts / kSpanPts);
  const int se = min(sb + kSegPts / kSpanPts, S) - 1;  // last span of the block
  const EntryRange er = entry_range(refl_offset, c, friedel);
  const int32_t *__restrict__ fs = span_first + c * span_cap;
  const int32_t *__restrict__ ls = span_last + c * span_cap;
  // entry ranges of the lane's spans (empty for spans past the grid's end)
  int f[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = sb + 16 * j + (int)(threadIdx.x / kSpanPts);
    f[j] = s <= se ? max(fs[s], 0) : 0;
    l[j] = s <= se ? (int)min((int64_t)ls[s], er.count - 1) : -1;
  }
  const int E0 = max(fs[sb], 0);
  const int E1 = (int)min((int64_t)ls[se], er.count - 1);
  double x[4];
  real acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[j] = g.t0 + (double)((int64_t)sb * kSpanPts + j * 256 + threadIdx.x) * g.dt;
    acc[j] = 0;
  }
  const real *__restrict__ wts = reinterpret_cast<const real *>(ent_w);
  const float c2 = (float)(g.inv2s2 * 1.4426950408889634);
  for (int T0 = E0; T0 <= E1; T0 += kGTile) {
    const int T1 = min(T0 + kGTile - 1, E1);
#pragma unroll
    for (int k = 0; k < kGTile / 256; ++k) {
      const int e = T0 + k * 256 + (int)threadIdx.x;
      if (e <= T1) {
        double2 v;
        v.x = ent_key[er.base + e];
        if constexpr (MIXED)
          v.y = __hiloint2double(0, __float_as_int(wts[er.base + e]));
        else
          v.y = wts[er.base + e];
        s_ent[e - T0] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = max(f[j], T0) - T0, b = min(l[j], T1) - T0;
      real sacc = acc[j];
#pragma unroll 4
      for (int e = a; e <= b; ++e) {
        const double2 ent = s_ent[e];
        const double d = x[j] - ent.x;
        if (fabs(d) <= g.half) {
          if constexpr (MIXED) {
            const float df = (float)d;
            const float w = __int_as_float(__double2loint(ent.y));
            sacc = __builtin_fmaf(w, __builtin_amdgcn_exp2f(-(df * df) * c2), sacc);
          } else {
            sacc += ent.y * exp(-(d * d) * g.inv2s2);
          }
        }
      }
      acc[j] = sacc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t p = (int64_t)sb * kSpanPts + j * 256 + threadIdx.x;
    if (p < g.n) y[c * g.n + p] = (double)acc[j];
  }
}

// Adjoint on the grid side, one block per kEntBlock consecutive entries of a
// crystal, four per thread (256 apart):
//   w1 = sum_g dy_g K,  w2 = sum_g dy_g K d / sigma^2  (d = x_g - 2theta)
// over the same window as the forward, K by the Gaussian recurrence (in
// single precision under MIXED, where 81-step products stay within ~1e-6).
// The block's entries are consecutive in 2theta, so their windows cover one
// interval of the grid; the block stages that stretch of the crystal's
// dL/dy row in LDS (converted to the working precision) when it has at most
// kAdjSpan points and reads the row from global memory otherwise.  Results
// go to (w1, w2) records at the entries' reflection indices (one 16-byte
// store each: the indices are scattered, so one store per record halves the
// partial-line writes).
template <typename real, typename src_t>
__device__ __forceinline__ void adj_walk(const src_t *__restrict__ src, int off, int wl, int wh, const GridArgs &g,
                                         double t, real rho, real dtr, real *a1o, real *a2o) {
#pragma clang fp contract(off)
  real a1 = 0, a2 = 0;
  if (wl <= wh) {
    const double d0 = g.t0 + (double)wl * g.dt - t;
    // the first kernel value and ratio: exponent arguments in double, the
    // exponentials in the working precision (single: v_exp_f32 of the
    // argument times log2 e)
    const double e0 = -(d0 * d0) * g.inv2s2, e1 = -(2.0 * d0 * g.dt + g.dt * g.dt) * g.inv2s2;
    real K, r;
    if constexpr (sizeof(real) == 4) {
      K = (real)g.norm * __builtin_amdgcn_exp2f((float)(e0 * 1.4426950408889634));
      r = __builtin_amdgcn_exp2f((float)(e1 * 1.4426950408889634));
    } else {
      K = (real)(g.norm * exp(e0));
      r = (real)exp(e1);
    }
    real d = (real)d0;
#pragma unroll 4
    for (int gi = wl; gi <= wh; ++gi) {
      const real kv = (real)src[gi - off] * K;
      a1 += kv;
      a2 = fma(kv, d, a2);
      K *= r;
      r *= rho;
      d += dtr;
    }
  }
  *a1o = a1;
  *a2o = a2;
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_broaden_adj(const HChunk *__restrict__ eblocks,
                                                     const CrystalPlan *__restrict__ plan, bool friedel,
                                                     const int64_t *__restrict__ refl_offset,
                                                     const double *__restrict__ ent_key,
                                                     const int32_t *__restrict__ ent_idx,
                                                     const double *__restrict__ dy, GridArgs g,
                                                     double2 *__restrict__ w12) {
#pragma clang fp contract(off)
  using real = typename std::conditional<MIXED, float, double>::type;
  __shared__ real s_dy[kAdjSpan];
  __shared__ int32_t s_span[2];
  constexpr int U = kEntBlock / 256;
  const HChunk hk = eblocks[blockIdx.x];
  const int32_t c = hk.crystal;
  const EntryRange er = entry_range(refl_offset, c, friedel);
  const int64_t e0 = (int64_t)hk.chunk * kEntBlock;
  if (e0 >= er.count) return;
  const int ne = (int)min((int64_t)kEntBlock, er.count - e0);
  double t[U];
  int32_t idx[U];
  int2 w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = u * 256 + (int)threadIdx.x;
    t[u] = ent_key[er.base + e0 + min(i, ne - 1)];
    idx[u] = i < ne ? ent_idx[er.base + e0 + i] : 0;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = u * 256 + (int)threadIdx.x;
    w[u] = window32(g, t[u]);
    // windows are nondecreasing in e: the block's stretch is [gl(first), gh(last)]
    if (i == 0) s_span[0] = w[u].x;
    if (i == ne - 1) s_span[1] = w[u].y;
  }
  __syncthreads();
  const int lo = s_span[0], hi = s_span[1];
  const double *__restrict__ dyc = dy + (int64_t)c * g.n;
  const double inv_s2 = 1.0 / (g.sigma * g.sigma);
  const real rho = (real)exp(-(g.dt * g.dt) * inv_s2);
  const real dtr = (real)g.dt;
  const bool staged = hi - lo + 1 <= kAdjSpan;
  if (staged) {
    const int len = hi - lo + 1;
#pragma unroll
    for (int k = 0; k < kAdjSpan / 256; ++k) {
      const int i = k * 256 + (int)threadIdx.x;
      if (i < len) s_dy[i] = (real)dyc[lo + i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = u * 256 + (int)threadIdx.x;
    if (i >= ne) continue;
    real a1, a2;
    if (staged)
      adj_walk<real, real>(s_dy, lo, w[u].x, w[u].y, g, t[u], rho, dtr, &a1, &a2);
    else
      adj_walk<real, double>(dyc, 0, w[u].x, w[u].y, g, t[u], rho, dtr, &a1, &a2);
    w12[idx[u]] = make_double2((double)a1, (double)a2 * inv_s2);
  }
}

GridArgs make_grid(double t0, double dt, int64_t n, double sigma, double window) {
  GridArgs g;
  g.t0 = t0;
  g.dt = dt;
  g.inv_dt = 1.0 / dt;
  g.n = n;
  g.sigma = sigma;
  g.half = window * sigma;
  g.norm = 1.0 / (sigma * sqrt(2.0 * kPi));
  g.inv2s2 = 1.0 / (2.0 * sigma * sigma);
  return g;
}

}  // namespace

void launch_broaden_fwd(bool mixed, const HChunk *eblocks, int64_t n_eblocks, const CrystalPlan *plan,
                        const int32_t *crystal_order, int64_t n_c, bool friedel, const int64_t *refl_offset, const double *ent_key,
                        const int32_t *ent_idx, const double *inten, double t0, double dt, int64_t n, double sigma,
                        double window, int64_t span_cap, double *ent_w, int32_t *span_first, int32_t *span_last,
                        double *y, hipStream_t s) {
  if (n_c <= 0 || n <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  if (n_eblocks > 0) {
    if (mixed)
      hipLaunchKernelGGL(k_entry_prep<true>, dim3((unsigned)n_eblocks), dim3(256), 0, s, eblocks,
                         plan, friedel, refl_offset, ent_key, ent_idx, inten, g, span_cap, ent_w, span_first,
                         span_last);
    else
      hipLaunchKernelGGL(k_entry_prep<false>, dim3((unsigned)n_eblocks), dim3(256), 0, s,
                         eblocks, plan, friedel, refl_offset, ent_key, ent_idx, inten, g, span_cap, ent_w,
                         span_first, span_last);
  }
  const dim3 grid((unsigned)(n_c * ((n + kSegPts - 1) / kSegPts))), block(256);
  if (mixed)
    hipLaunchKernelGGL(k_broaden_gather<true>, grid, block, 0, s, crystal_order, refl_offset, friedel, ent_key, ent_w,
                       span_first, span_last, span_cap, g, y);
  else
    hipLaunchKernelGGL(k_broaden_gather<false>, grid, block, 0, s, crystal_order, refl_offset, friedel, ent_key,
                       ent_w, span_first, span_last, span_cap, g, y);
}

void launch_broaden_adj(bool mixed, const HChunk *eblocks, int64_t n_eblocks, const CrystalPlan *plan,
                        bool friedel, const int64_t *refl_offset, const double *ent_key, const int32_t *ent_idx,
                        const double *dy, double t0, double dt, int64_t n, double sigma, double window,
                        double2 *w12, hipStream_t s) {
  if (n_eblocks <= 0 || n <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  const dim3 grid((unsigned)n_eblocks), block(256);
  if (mixed)
    hipLaunchKernelGGL(k_broaden_adj<true>, grid, block, 0, s, eblocks, plan, friedel, refl_offset, ent_key,
                       ent_idx, dy, g, w12);
  else
    hipLaunchKernelGGL(k_broaden_adj<false>, grid, block, 0, s, eblocks, plan, friedel, refl_offset, ent_key,
                       ent_idx, dy, g, w12);
}


}  // namespace xrd
