// Experimental effects for ML training patterns (paper, Section 1: the
// simulated patterns of ML training sets are modified with effects such as
// preferred orientation and noise).
//
// Preferred orientation (March-Dollase, Dollase, J. Appl. Cryst. 19 (1986)
// 267): each reflection's intensity is multiplied by
//   P = (r^2 cos^2(alpha) + sin^2(alpha) / r)^(-3/2),
//   cos(alpha) = h^T G* hp / (|h| |hp|),  |v| = sqrt(v^T G* v),
// for the crystal's preferred direction hp (a reciprocal-lattice vector in
// hkl components) and March parameter r.  Every hkl is enumerated on its
// own, so the factor applies per reflection with no average over families.
//
// Noise: y += (rel sqrt(max(y, 0)) + abs) z at every grid point, z the
// standard normal variate number (c n_points + g) of the stream ``seed``:
// outputs 2n+1 and 2n+2 of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
// give two uniforms in (0, 1) (top 53 bits plus one half, times 2^-53), and
// the Box-Muller transform sqrt(-2 ln u1) cos(2 pi u2) gives z.  A counter
// rather than a sequential state, so every point draws its own variate in
// parallel and a seed fixes the result.
//
// Peak widths that grow with angle (Caglioti, Paoletti and Ricci, Nucl.
// Instrum. 3 (1958) 223): the broadened pattern with FWHM^2 = U tan^2(theta)
// + V tan(theta) + W per reflection instead of one width, and pseudo-Voigt
// profiles eta L + (1 - eta) G: a unit-area Lorentzian and a unit-area
// Gaussian of that FWHM, both cut at the window.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double dot_gs(const double *__restrict__ gs, const double u0, const double u1,
                                         const double u2, const double v0, const double v1, const double v2) {
  return gs[0] * u0 * v0 + gs[1] * u1 * v1 + gs[2] * u2 * v2 + gs[3] * (u0 * v1 + u1 * v0) +
         gs[4] * (u0 * v2 + u2 * v0) + gs[5] * (u1 * v2 + u2 * v1);
}

// One block per (crystal, chunk of kSortChunk reflection slots) of the peak
// chunk table, which covers every crystal's reflection capacity; four
// reflections per thread.
__global__ __launch_bounds__(kThreads) void k_march_dollase(const HChunk *__restrict__ chunks,
                                                            const CrystalPlan *__restrict__ plan,
                                                            const int64_t *__restrict__ refl_offset,
                                                            const int16_t *__restrict__ hh,
                                                            const int16_t *__restrict__ kk,
                                                            const int16_t *__restrict__ ll,
                                                            const double *__restrict__ hp,
                                                            const double *__restrict__ march_r,
                                                            double *__restrict__ inten) {
  const HChunk ch = chunks[blockIdx.x];
  const int64_t c = ch.crystal;
  const int64_t r1 = refl_offset[c + 1];
  const int64_t i0 = refl_offset[c] + (int64_t)ch.chunk * kSortChunk;
  if (i0 >= r1) return;
  const double r = march_r[c], p0 = hp[3 * c], p1 = hp[3 * c + 1], p2 = hp[3 * c + 2];
  const double *gs = plan[c].gs;
  const double pp = dot_gs(gs, p0, p1, p2, p0, p1, p2);
  if (!(r > 0.0) || !(pp > 0.0)) return;  // no texture for this crystal
  const double r2 = r * r, inv_r = 1.0 / r;
#pragma unroll
  for (int u = 0; u < kSortChunk / kThreads; ++u) {
    const int64_t i = i0 + u * kThreads + threadIdx.x;
    if (i < r1) {
      const double h = hh[i], k = kk[i], l = ll[i];
      const double ca = dot_gs(gs, h, k, l, p0, p1, p2) / sqrt(dot_gs(gs, h, k, l, h, k, l) * pp);
      const double c2 = ca * ca;
      const double x = r2 * c2 + (1.0 - c2) * inv_r;
      inten[i] *= 1.0 / (x * sqrt(x));  // x^(-3/2)
    }
  }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + j * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kThreads) void k_noise(int64_t total, uint64_t seed, double rel, double abs_,
                                                    double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
    const uint64_t n = (uint64_t)i;
    const double u1 = ((double)(splitmix64(seed, 2 * n + 1) >> 11) + 0.5) * 0x1p-53;
    const double u2 = ((double)(splitmix64(seed, 2 * n + 2) >> 11) + 0.5) * 0x1p-53;
    const double z = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    const double v = y[i];
    y[i] = v + (rel * sqrt(v > 0.0 ? v : 0.0) + abs_) * z;
  }
}

// Smallest i in [0, n] with keys[i] >= target (STRICT: keys[i] > target), or
// n, for keys sorted ascending; every thread of the block calls it.  Each
// round samples the remaining range at 256 evenly spaced positions and keeps
// the stretch between the last sample below the target and the first one
// above it, so a range of n keys takes about log_256(n) rounds.
template <bool STRICT>
__device__ int64_t block_lower_bound(const double *__restrict__ keys, int64_t n, double target) {
  int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
  while (hi > lo) {
    const int64_t stride = (hi - lo + kThreads - 1) / kThreads;
    const int64_t i = lo + (int64_t)threadIdx.x * stride;
    const bool below = i < hi && (STRICT ? !(keys[i] > target) : keys[i] < target);
    const int nb = __syncthreads_count(below);  // the samples below form a prefix
    if (nb == 0) {
      hi = lo;
    } else {
      const int64_t last = lo + (int64_t)(nb - 1) * stride;  // below the target
      hi = min(hi, last + stride);
      lo = last + 1;
    }
  }
  return lo;
}

// Gaussian broadening with Caglioti widths, FWHM^2 = U tan^2(theta) +
// V tan(theta) + W (degrees^2), sigma = FWHM / (2 sqrt(2 ln 2)), over the
// points with |x - 2theta| <= window sigma; entries with FWHM^2 <= 0 add
// nothing.  A block owns 256 consecutive grid points of one crystal (a thread
// each): it finds the entries within the largest half-width of its points
// (the crystal's widest line, from the width's maximum over its 2theta
// range) by two searches over the sorted entries, stages them 256 at a time
// in LDS with their weight, exponent scale and half-width, and every thread
// sums its lines in 2theta order, in double precision.  Under MIXED the
// Gaussian itself is the single-precision exp2 of -d^2 log2(e) / (2 sigma^2)
// with d = x - 2theta rounded to single after the double subtraction (about
// 4e-6 relative per term at the window's edge, less nearer the centre), as in
// the constant-width gather; otherwise exp in double.
struct CagEnt {
  double t, w;   // 2theta, (1 - eta) intensity / (sigma sqrt(2 pi)) (0: no line)
  double z;      // 1 / (2 sigma^2), times log2(e) under MIXED
  double half;   // window * sigma (-1: no line)
  double wl;     // eta intensity 2 / (pi FWHM): the Lorentzian's peak
  double ql;     // (2 / FWHM)^2
};

// Logical block of a launch of g blocks such that consecutive logical blocks
// share an XCD: workgroups go to the eight XCDs round-robin by blockIdx, and
// each XCD has its own L2, so neighbouring work (one crystal's blocks) should
// land on one of them.  A bijection of [0, g): XCD x (= blockIdx mod 8) takes
// a contiguous range of logical blocks, ceil(g / 8) or one fewer.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t g) {
  constexpr int64_t kXcd = 8;
  const int64_t per = (g + kXcd - 1) / kXcd, tall = g - (per - 1) * kXcd;  // XCDs taking ``per`` blocks
  const int64_t x = b % kXcd, i = b / kXcd;
  return x < tall ? x * per + i : tall * per + (x - tall) * (per - 1) + i;
}

template <bool MIXED>
__global__ __launch_bounds__(kThreads) void k_broaden_caglioti(
    const CrystalPlan *__restrict__ plan, const int64_t *__restrict__ refl_offset, bool friedel,
    const double *__restrict__ ent_key, const int32_t *__restrict__ ent_idx, const double *__restrict__ inten,
    double t0, double dt, int64_t n, double U, double V, double W, double eta, double window,
    double *__restrict__ y) {
  __shared__ CagEnt s_ent[kThreads];
  const int64_t blocks_per = (n + kThreads - 1) / kThreads;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t c = lb / blocks_per;
  const int64_t p = (lb % blocks_per) * kThreads + threadIdx.x;
  const CrystalPlan &P = plan[c];
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  const int64_t base = friedel ? r0 / 2 : r0, count = friedel ? (r1 - r0) / 2 : r1 - r0;
  const double m = friedel ? 2.0 : 1.0;
  const double rad = 3.14159265358979323846 / 360.0;  // degrees of 2theta to radians of theta
  const double fw = 1.0 / (2.0 * sqrt(2.0 * log(2.0)));
  // the widest line of the crystal: FWHM^2 is a quadratic in tan(theta), so
  // its maximum over the crystal's range lies at an end or at the vertex
  const double ta = tan(P.tmin * rad), tb = tan(P.tmax * rad);
  auto f2 = [&](double t) { return (U * t + V) * t + W; };
  double f2max = fmax(f2(ta), f2(tb));
  if (U < 0.0) {
    const double tv = -V / (2.0 * U);
    if (tv > ta && tv < tb) f2max = fmax(f2max, f2(tv));
  }
  const double hmax = f2max > 0.0 ? window * sqrt(f2max) * fw : 0.0;
  const int64_t p0 = (lb % blocks_per) * kThreads;
  const int64_t p1 = min(p0 + kThreads, n) - 1;
  const double x0 = t0 + (double)p0 * dt, x1 = t0 + (double)p1 * dt;
  const double *keys = ent_key + base;
  const int64_t e0 = block_lower_bound<false>(keys, count, x0 - hmax);
  const int64_t e1 = block_lower_bound<true>(keys, count, x1 + hmax);
  const double x = t0 + (double)p * dt;
  const int lane = threadIdx.x & 63;
  const int64_t pw0 = p0 + (threadIdx.x & ~63), pw1 = min(pw0 + 64, n) - 1;
  const double xw_lo = t0 + (double)pw0 * dt - hmax, xw_hi = t0 + (double)max(pw1, pw0) * dt + hmax;
  double acc = 0.0;
  for (int64_t t0e = e0; t0e < e1; t0e += kThreads) {
    const int64_t e = t0e + threadIdx.x;
    __syncthreads();  // the previous tile has been read
    if (e < e1) {
      const double t = keys[e];
      const double tn = tan(t * rad);
      const double q = f2(tn);
      CagEnt v{t, 0.0, 0.0, -1.0, 0.0, 0.0};
      if (q > 0.0) {
        const double gam = sqrt(q), sigma = gam * fw;
        const double mi = m * inten[ent_idx[base + e]];
        v.w = (1.0 - eta) * mi / (sigma * sqrt(2.0 * 3.14159265358979323846));
        v.z = 1.0 / (2.0 * sigma * sigma);
        if constexpr (MIXED) v.z *= 1.44269504088896340736;  // log2(e)
        v.half = window * sigma;
        v.wl = eta * mi * 2.0 / (3.14159265358979323846 * gam);
        v.ql = 4.0 / q;
      }
      s_ent[threadIdx.x] = v;
    }
    __syncthreads();
    const int ne = (int)min((int64_t)kThreads, e1 - t0e);
    // the wavefront's own stretch of the sorted tile: entries within hmax of
    // its 64 points (counted by ballots; the rest cannot reach them)
    int j0 = 0, j1 = 0;
#pragma unroll
    for (int q = 0; q < kThreads; q += 64) {
      const int j = q + lane;
      const bool in = j < ne;
      const double t = in ? s_ent[j].t : 0.0;
      j0 += __popcll(__ballot(in && t < xw_lo));
      j1 += __popcll(__ballot(in && !(t > xw_hi)));
    }
    if (eta == 0.0) {
      for (int j = j0; j < j1; ++j) {
        const CagEnt v = s_ent[j];
        const double d = x - v.t;
        if (fabs(d) <= v.half) {
          if constexpr (MIXED) {
            const float df = (float)d;
            acc = fma(v.w, (double)__builtin_amdgcn_exp2f(-(df * df) * (float)v.z), acc);
          } else {
            acc += v.w * exp(-(d * d) * v.z);
          }
        }
      }
    } else {
      for (int j = j0; j < j1; ++j) {
        const CagEnt v = s_ent[j];
        const double d = x - v.t;
        if (fabs(d) <= v.half) {
          if constexpr (MIXED) {
            const float df = (float)d, d2 = df * df;
            const float g = __builtin_amdgcn_exp2f(-d2 * (float)v.z);
            const float lz = __builtin_amdgcn_rcpf(fmaf(d2, (float)v.ql, 1.0f));
            acc = fma(v.w, (double)g, fma(v.wl, (double)lz, acc));
          } else {
            acc += v.wl / (1.0 + (d * d) * v.ql) + v.w * exp(-(d * d) * v.z);
          }
        }
      }
    }
  }
  if (p < n) y[c * n + p] = acc;
}

}  // namespace

void launch_broaden_caglioti(bool mixed, const CrystalPlan *plan, int64_t n_c, const int64_t *refl_offset,
                             bool friedel, const double *ent_key, const int32_t *ent_idx, const double *inten,
                             double t0, double dt, int64_t n, double U, double V, double W, double eta, double window,
                             double *y, hipStream_t s) {
  if (n_c <= 0 || n <= 0) return;
  const int64_t blocks = n_c * ((n + kThreads - 1) / kThreads);
  if (mixed)
    hipLaunchKernelGGL(k_broaden_caglioti<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, plan, refl_offset,
                       friedel, ent_key, ent_idx, inten, t0, dt, n, U, V, W, eta, window, y);
  else
    hipLaunchKernelGGL(k_broaden_caglioti<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, plan, refl_offset,
                       friedel, ent_key, ent_idx, inten, t0, dt, n, U, V, W, eta, window, y);
}

void launch_march_dollase(const HChunk *chunks, int64_t n_chunks, const CrystalPlan *plan,
                          const int64_t *refl_offset, const int16_t *h, const int16_t *k, const int16_t *l,
                          const double *hp, const double *march_r, double *inten, hipStream_t s) {
  if (n_chunks <= 0) return;
  hipLaunchKernelGGL(k_march_dollase, dim3((unsigned)n_chunks), dim3(kThreads), 0, s, chunks, plan, refl_offset, h, k,
                     l, hp, march_r, inten);
}

void launch_noise(int64_t total, uint64_t seed, double rel, double abs_, double *y, hipStream_t s) {
  if (total <= 0) return;
  const int64_t blocks = (total + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_noise, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kThreads), 0, s, total, seed,
                     rel, abs_, y);
}

}  // namespace xrd
