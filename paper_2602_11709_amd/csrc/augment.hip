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

}  // namespace

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
