// Gaussian broadening of the reflections onto a 2theta grid, and the grid side
// of its adjoint.  The paper motivates fast simulation with machine-learning
// datasets of patterns modified by peak broadening (Section 1); this is the
// differentiable pattern those models consume.
//
//   y_g = sum_r I_r K(x_g - 2theta_r),  K(d) = exp(-d^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
//   restricted to |x_g - 2theta_r| <= window * sigma, x_g = t0 + g dt.
//
// Forward: a gather in which each thread owns one grid point and sums, in
// 2theta order, the reflections staged in LDS whose window holds it, so the
// result is deterministic without atomics.  Adjoint: per evaluated
// reflection, w1 = sum_g dL/dy_g K and w2 = sum_g dL/dy_g K (x_g - 2theta) /
// sigma^2 over the same window; on the uniform grid the Gaussian follows a
// two-term multiplicative recurrence, so a whole window costs two exp and a
// few products per point.  Then the lattice chain rule of the per-crystal
// dL/dG*.
#include <math.h>

#include <type_traits>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GridArgs {
  double t0, dt, sigma, half, norm, inv2s2;
  int64_t n;
};

// Grid points covered by a reflection at 2theta t: the interval of g in
// [0, n) with |x_g - t| <= half, x_g = t0 + g dt (an interval because x_g - t
// is monotone in g).  Empty when lo > hi.
__device__ __forceinline__ void window_of(const GridArgs &g, double t, int64_t *lo, int64_t *hi) {
#pragma clang fp contract(off)
  int64_t a = (int64_t)ceil((t - g.half - g.t0) / g.dt);
  int64_t b = (int64_t)floor((t + g.half - g.t0) / g.dt);
  // the estimates are off by at most one step either way; settle them with the exact test
  while (a > 0 && fabs(g.t0 + (double)(a - 1) * g.dt - t) <= g.half) --a;
  while (a <= b && fabs(g.t0 + (double)a * g.dt - t) > g.half) ++a;
  while (b + 1 < g.n && fabs(g.t0 + (double)(b + 1) * g.dt - t) <= g.half) ++b;
  while (b >= a && fabs(g.t0 + (double)b * g.dt - t) > g.half) --b;
  if (a < 0) a = 0;
  if (b > g.n - 1) b = g.n - 1;
  *lo = a;
  *hi = b;
}

// Gaussian values along the grid by recurrence: with d = x_g - t,
// K(d + dt) = K(d) r(d), r(d) = exp(-(2 d dt + dt^2) / (2 sigma^2)) and
// r(d + dt) = r(d) rho, rho = exp(-dt^2 / sigma^2); two exp per window.
struct GaussWalk {
  double K, r;
  __device__ __forceinline__ void start(const GridArgs &g, double d, double scale) {
    K = scale * g.norm * exp(-(d * d) * g.inv2s2);
    r = exp(-(2.0 * d * g.dt + g.dt * g.dt) * g.inv2s2);
  }
  __device__ __forceinline__ void step(double rho) {
    K *= r;
    r *= rho;
  }
};

constexpr int kPtsPerThread = 4;
constexpr int kSegPts = 256 * kPtsPerThread;  // grid points per block of the forward gather
constexpr int kTileR = 1024;                  // reflections per LDS tile of the gather
constexpr int kAdjDyLds = 8192;               // grid rows up to this length are staged in LDS by the adjoint
constexpr int kAdjSplit = 4;                  // adjoint blocks per chunk of evaluated reflections

// First position in [lo, hi) of a sorted array with a[i] >= v, searched by the
// whole block: each level probes 256 evenly spaced positions with one load
// per thread and counts the probes below v, so a level shrinks the range
// 256-fold (two levels for a crystal of up to 65536 reflections).  Every
// thread of the block must call it.
__device__ __forceinline__ int64_t block_lower_bound(const double *__restrict__ a, int64_t lo, int64_t hi, double v) {
  int64_t base = lo, len = hi - lo;
  while (len > 0) {
    const int64_t stride = (len + 255) / 256;
    const int64_t p = base + (int64_t)threadIdx.x * stride;
    const bool below = p < base + len && a[p] < v;
    const int cnt = __syncthreads_count(below);
    if (cnt == 0) return base;
    const int64_t nb = base + (int64_t)(cnt - 1) * stride + 1;
    const int64_t ne = min(base + (int64_t)cnt * stride, base + len);
    base = nb;
    len = ne - nb;
  }
  return base;
}

// Forward gather.  A block owns kSegPts consecutive grid points of one
// crystal; each thread kPtsPerThread of them, 256 apart.  The crystal's
// 2theta-sorted reflections that reach the block's points are staged through
// LDS in tiles (with Friedel pairing, whose mates have bit-identical 2theta
// and I, one reflection per pair with twice the intensity), each with its
// exact grid window [gl, gh] (the points with |x - 2theta| <= half).  Windows
// are ordered like 2theta, so the reflections reaching point p form a range
// [first e with gh_e >= p, last e with gl_e <= p]; both ends are scattered
// into per-point LDS arrays, and every point then sums its range in sorted
// order with no data-dependent exit: deterministic, no atomics.  The kernel
// value is exp(-d^2 / 2 sigma^2) with d = x - 2theta in double; under MIXED
// the exponential is taken in single precision (v_exp_f32).
template <bool MIXED>
__global__ __launch_bounds__(256) void k_broaden_fwd(const int64_t *__restrict__ refl_offset,
                                                     const double *__restrict__ skey,
                                                     const int32_t *__restrict__ sidx,
                                                     const double *__restrict__ inten, GridArgs g, bool friedel,
                                                     double *__restrict__ y) {
#pragma clang fp contract(off)
  __shared__ double s_tt[kTileR], s_i[kTileR];
  __shared__ int32_t s_gl[kTileR], s_gh[kTileR];
  __shared__ int16_t s_first[kSegPts], s_last[kSegPts];
  __shared__ int32_t s_wcnt[256 / 64];
  const int64_t segs = (g.n + kSegPts - 1) / kSegPts;
  const int64_t c = blockIdx.x / segs;
  const int64_t G0 = (int64_t)(blockIdx.x % segs) * kSegPts;
  const int64_t G1 = min(G0 + kSegPts, g.n) - 1;
  const int npts = (int)(G1 - G0 + 1);
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  const int64_t mid = r0 + (r1 - r0) / 2;  // first reflection of the positive half
  const double xa = g.t0 + (double)G0 * g.dt, xb = g.t0 + (double)G1 * g.dt;
  const double bguard = 1e-9 * (fabs(xa) + fabs(xb) + 1.0);
  const int64_t ja = block_lower_bound(skey, r0, r1, xa - g.half - bguard);
  const int64_t jb = block_lower_bound(skey, ja, r1, xb + g.half + bguard);
  const float c2 = (float)(g.inv2s2 * 1.4426950408889634);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double acc[kPtsPerThread], x[kPtsPerThread];
#pragma unroll
  for (int q = 0; q < kPtsPerThread; ++q) {
    acc[q] = 0.0;
    x[q] = g.t0 + (double)(G0 + q * 256 + threadIdx.x) * g.dt;
  }
  for (int64_t jt = ja; jt < jb; jt += kTileR) {
    // stage in sorted order, compacted with a ballot per wave
    int base = 0;
    const int rounds = (int)min((int64_t)(kTileR / 256), (jb - jt + 255) / 256);
    for (int u = 0; u < rounds; ++u) {
      const int64_t j = jt + u * 256 + threadIdx.x;
      bool keep = j < jb;
      int32_t id = 0;
      if (keep) {
        id = sidx[j];
        keep = !friedel || id >= mid;
      }
      const uint64_t bal = __ballot(keep);
      if (lane == 0) s_wcnt[wid] = __popcll(bal);
      __syncthreads();
      int before = 0, total = 0;
      for (int w = 0; w < 256 / 64; ++w) {
        before += w < wid ? s_wcnt[w] : 0;
        total += s_wcnt[w];
      }
      if (keep) {
        const int e = base + before +
                      __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        const double t = skey[j];
        int64_t wl, wh;
        window_of(g, t, &wl, &wh);
        s_tt[e] = t;
        s_i[e] = (friedel ? 2.0 : 1.0) * inten[id] * g.norm;
        // window relative to the segment, clamped to [-1, npts]
        s_gl[e] = (int32_t)max((int64_t)-1, min((int64_t)npts, wl - G0));
        s_gh[e] = (int32_t)max((int64_t)-1, min((int64_t)npts, wh - G0));
      }
      base += total;
      __syncthreads();
    }
    const int nt = base;
    // per point: first entry with gh >= p and last entry with gl <= p (empty: last < first)
    for (int p = threadIdx.x; p < npts; p += 256) {
      s_first[p] = (int16_t)nt;
      s_last[p] = (int16_t)-1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt; e += 256) {
      // points p in (gh_{e-1}, gh_e] have first = e; points in [gl_e, gl_{e+1}) have last = e
      const int ghp = e ? s_gh[e - 1] : -1, gh = s_gh[e];
      for (int p = max(ghp + 1, 0); p <= min(gh, npts - 1); ++p) s_first[p] = (int16_t)e;
      const int gl = s_gl[e], gln = e + 1 < nt ? s_gl[e + 1] : npts;
      for (int p = max(gl, 0); p < min(gln, npts); ++p) s_last[p] = (int16_t)e;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPtsPerThread; ++q) {
      const int p = q * 256 + threadIdx.x;
      if (p >= npts) continue;
      const int e0 = s_first[p], e1 = s_last[p];
      double a = 0.0;
      for (int e = e0; e <= e1; ++e) {
        const double d = x[q] - s_tt[e];
        if constexpr (MIXED) {
          const float df = (float)d;
          a += s_i[e] * (double)__builtin_amdgcn_exp2f(-(df * df) * c2);
        } else {
          a += s_i[e] * exp(-(d * d) * g.inv2s2);
        }
      }
      acc[q] += a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPtsPerThread; ++q) {
    const int64_t gi = G0 + q * 256 + threadIdx.x;
    if (gi <= G1) y[c * g.n + gi] = acc[q];
  }
}

// Adjoint on the grid side: kAdjSplit blocks per chunk of a crystal's
// evaluated reflections, the crystal's dL/dy row staged in LDS; per reflection
//   w1 = sum_g dy_g K,  w2 = sum_g dy_g K d / sigma^2  (d = x_g - 2theta)
// over the same window as the forward, K by the Gaussian recurrence (in
// single precision under MIXED, where 81-step products stay within ~1e-6).
template <bool LDS_ROW, bool MIXED>
__global__ __launch_bounds__(256) void k_broaden_adj(const int32_t *__restrict__ hchunk_crystal,
                                                     const CrystalPlan *__restrict__ plan, bool friedel,
                                                     const int64_t *__restrict__ refl_offset,
                                                     const double *__restrict__ tt, const double *__restrict__ dy,
                                                     GridArgs g, double *__restrict__ w1, double *__restrict__ w2) {
#pragma clang fp contract(off)
  using real = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ double s_dy[];  // the crystal's dL/dy row when LDS_ROW
  const int hc = blockIdx.x / kAdjSplit, sub = blockIdx.x % kAdjSplit;
  const int32_t c = hchunk_crystal[hc];
  const CrystalPlan &P = plan[c];
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  const int64_t first = friedel ? r0 + (r1 - r0) / 2 : r0;
  const int64_t count = friedel ? (r1 - r0) / 2 : r1 - r0;
  const int64_t e0 = (int64_t)(hc - P.hchunk_begin) * kHalfChunk + sub * (kHalfChunk / kAdjSplit);
  if (e0 >= count) return;
  const int64_t e1 = min(e0 + (int64_t)(kHalfChunk / kAdjSplit), count);
  const double *dyc = dy + (int64_t)c * g.n;
  if (LDS_ROW) {
    for (int i = threadIdx.x; i < (int)g.n; i += 256) s_dy[i] = dyc[i];
    __syncthreads();
  }
  const double inv_s2 = 1.0 / (g.sigma * g.sigma);
  const real rho = (real)exp(-(g.dt * g.dt) * inv_s2);
  const real dtr = (real)g.dt;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int64_t i = first + e;
    const double t = tt[i];
    int64_t wl64, wh64;
    window_of(g, t, &wl64, &wh64);
    const int wl = (int)wl64, wh = (int)wh64;
    real a1 = 0, a2 = 0;
    if (wl <= wh) {
      const double d0 = g.t0 + (double)wl * g.dt - t;
      real K = (real)(g.norm * exp(-(d0 * d0) * g.inv2s2));
      real r = (real)exp(-(2.0 * d0 * g.dt + g.dt * g.dt) * g.inv2s2);
      real d = (real)d0;
      for (int gi = wl; gi <= wh; ++gi) {
        const real kv = (real)(LDS_ROW ? s_dy[gi] : dyc[gi]) * K;
        a1 += kv;
        a2 += kv * d;
        K *= r;
        r *= rho;
        d += dtr;
      }
    }
    w1[i] = (double)a1;
    w2[i] = (double)a2 * inv_s2;
  }
}

// dL/dG* (6 unique entries) -> dL/d(a, b, c, alpha, beta, gamma), angles in degrees.
// q = sum_ij M_ij h_i h_j with M = G*, so dL/dM_ij = U_ij for i == j and
// U_ij / 2 for i != j (the unique entry appears twice); dL/dG = -M (dL/dM) M.
__global__ void k_lattice_chain(const CrystalPlan *__restrict__ plan, int64_t n_c, const double *__restrict__ part6,
                                double *__restrict__ dlat) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_c) return;
  const CrystalPlan &P = plan[c];
  double U[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < P.n_hchunks; ++k)
    for (int e = 0; e < 6; ++e) U[e] += part6[(P.hchunk_begin + k) * 6 + e];
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
  const double rad = kPi / 180.0;
  double sa, ca, sb, cb, sg, cg;
  sincos(P.lat[3] * rad, &sa, &ca);
  sincos(P.lat[4] * rad, &sb, &cb);
  sincos(P.lat[5] * rad, &sg, &cg);
  // G11 = a^2, G22 = b^2, G33 = c^2, G12 = ab cos(gamma), G13 = ac cos(beta), G23 = bc cos(alpha);
  // off-diagonal entries appear twice in the full symmetric matrix.
  const double g12 = 2.0 * Gb[0][1], g13 = 2.0 * Gb[0][2], g23 = 2.0 * Gb[1][2];
  double *o = dlat + 6 * c;
  o[0] = Gb[0][0] * 2.0 * a + g12 * b * cg + g13 * cc * cb;
  o[1] = Gb[1][1] * 2.0 * b + g12 * a * cg + g23 * cc * ca;
  o[2] = Gb[2][2] * 2.0 * cc + g13 * a * cb + g23 * b * ca;
  o[3] = g23 * (-b * cc * sa * rad);
  o[4] = g13 * (-a * cc * sb * rad);
  o[5] = g12 * (-a * b * sg * rad);
}

GridArgs make_grid(double t0, double dt, int64_t n, double sigma, double window) {
  GridArgs g;
  g.t0 = t0;
  g.dt = dt;
  g.n = n;
  g.sigma = sigma;
  g.half = window * sigma;
  g.norm = 1.0 / (sigma * sqrt(2.0 * kPi));
  g.inv2s2 = 1.0 / (2.0 * sigma * sigma);
  return g;
}

}  // namespace

void launch_broaden_fwd(bool mixed, int64_t n_c, const int64_t *refl_offset, const double *skey,
                        const int32_t *sidx, const double *inten, bool friedel, double t0, double dt, int64_t n,
                        double sigma, double window, double *y, hipStream_t s) {
  if (n_c <= 0 || n <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  const int64_t segs = (n + kSegPts - 1) / kSegPts;
  if (mixed)
    hipLaunchKernelGGL(k_broaden_fwd<true>, dim3((unsigned)(segs * n_c)), dim3(256), 0, s, refl_offset, skey, sidx,
                       inten, g, friedel, y);
  else
    hipLaunchKernelGGL(k_broaden_fwd<false>, dim3((unsigned)(segs * n_c)), dim3(256), 0, s, refl_offset, skey, sidx,
                       inten, g, friedel, y);
}

void launch_broaden_adj(bool mixed, const int32_t *hchunk_crystal, int64_t n_hchunks, const CrystalPlan *plan,
                        bool friedel, const int64_t *refl_offset, const double *tt, const double *dy, double t0,
                        double dt, int64_t n, double sigma, double window, double *w1, double *w2, hipStream_t s) {
  if (n_hchunks <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  const dim3 grid((unsigned)(n_hchunks * kAdjSplit)), block(256);
  const size_t lds = (size_t)n * sizeof(double);
  if (n <= kAdjDyLds) {
    if (mixed)
      hipLaunchKernelGGL((k_broaden_adj<true, true>), grid, block, lds, s, hchunk_crystal, plan, friedel, refl_offset,
                         tt, dy, g, w1, w2);
    else
      hipLaunchKernelGGL((k_broaden_adj<true, false>), grid, block, lds, s, hchunk_crystal, plan, friedel,
                         refl_offset, tt, dy, g, w1, w2);
  } else {
    if (mixed)
      hipLaunchKernelGGL((k_broaden_adj<false, true>), grid, block, 0, s, hchunk_crystal, plan, friedel, refl_offset,
                         tt, dy, g, w1, w2);
    else
      hipLaunchKernelGGL((k_broaden_adj<false, false>), grid, block, 0, s, hchunk_crystal, plan, friedel,
                         refl_offset, tt, dy, g, w1, w2);
  }
}

void launch_lattice_chain(const CrystalPlan *plan, int64_t n_c, const double *part6, double *dlat, hipStream_t s) {
  if (n_c <= 0) return;
  hipLaunchKernelGGL(k_lattice_chain, dim3((unsigned)((n_c + 255) / 256)), dim3(256), 0, s, plan, n_c, part6, dlat);
}

}  // namespace xrd
