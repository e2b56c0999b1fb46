// Peaks of two emission lines of the same crystals in one list per crystal
// (paper, Section 2: the calculator's peaks with their 2theta, intensity,
// interplanar spacing and multiplicity, scaled to 0-100 on request; the
// K-alpha1/K-alpha2 doublet is computed as two lines whose peaks are listed
// side by side and scaled together).
//
// kSplit blocks per crystal (each takes every kSplit-th stretch of kThreads
// peaks and computes the crystal's maximum itself).  Each line's peaks are
// already in ascending 2theta, so a peak's slot in the combined list is its
// index in its own list plus the number of the other line's peaks before it
// (binary search; at equal 2theta the first line's peaks come first).  The crystal's combined offset is the
// sum of the two lines' offsets, so no scan is needed.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int kSplit = 8;  // blocks per crystal

// Number of elements of the ascending a[0, n) below t (strict) or at most t.
template <bool INCLUSIVE>
__device__ __forceinline__ int64_t rank_in(const double *__restrict__ a, int64_t n, double t) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const bool before = INCLUSIVE ? a[mid] <= t : a[mid] < t;
    if (before)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

struct LineIn {
  const double *tt, *inten, *q;
  const int32_t *mult;
  const int64_t *first, *perm, *offset;
  double weight;
};

__device__ void place_line(const LineIn &me, const LineIn &other, bool second, int64_t a, int64_t b, int64_t oa,
                           int64_t ob, int64_t o, double mx, int line, const LineOut &out) {
  const int64_t n_other = ob - oa;
  for (int64_t i = a + (int64_t)blockIdx.y * kThreads + threadIdx.x; i < b; i += (int64_t)kSplit * kThreads) {
    const double t = me.tt[i];
    // the first line's peaks precede the second's at equal 2theta
    const int64_t r = second ? rank_in<true>(other.tt + oa, n_other, t) : rank_in<false>(other.tt + oa, n_other, t);
    const int64_t k = o + (i - a) + r;
    const double y = me.weight * me.inten[i];
    out.two_theta[k] = t;
    out.intensity[k] = y;
    out.scaled[k] = mx > 0.0 ? 100.0 * y / mx : 0.0;
    out.mult[k] = me.mult[i];
    out.d[k] = 1.0 / sqrt(me.q[me.perm[me.first[i]]]);
    out.line[k] = line;
    out.source[k] = i;
  }
}

__global__ __launch_bounds__(kThreads) void k_combine_lines(int64_t n_c, LineIn l0, LineIn l1, bool two,
                                                            LineOut out) {
  __shared__ double red[kThreads / 64];
  const int64_t c = blockIdx.x;
  const int64_t a0 = l0.offset[c], b0 = l0.offset[c + 1];
  const int64_t a1 = two ? l1.offset[c] : 0, b1 = two ? l1.offset[c + 1] : 0;
  // the crystal's largest weighted intensity over both lines
  double mx = 0.0;
  for (int64_t i = a0 + threadIdx.x; i < b0; i += kThreads) mx = fmax(mx, l0.weight * l0.inten[i]);
  for (int64_t i = a1 + threadIdx.x; i < b1; i += kThreads) mx = fmax(mx, l1.weight * l1.inten[i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mx = fmax(mx, __shfl_xor(mx, d, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) mx = fmax(mx, red[w]);
  const int64_t o = a0 + a1;
  place_line(l0, l1, false, a0, b0, a1, b1, o, mx, 0, out);
  if (two) place_line(l1, l0, true, a1, b1, a0, b0, o, mx, 1, out);
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    out.peak_offset[c] = o;
    if (c == n_c - 1) out.peak_offset[n_c] = l0.offset[n_c] + (two ? l1.offset[n_c] : 0);
  }
}

LineIn line_in(const LinePeaks &p) {
  LineIn l;
  l.tt = p.two_theta;
  l.inten = p.intensity;
  l.q = p.q;
  l.mult = p.mult;
  l.first = p.first;
  l.perm = p.perm;
  l.offset = p.peak_offset;
  l.weight = p.weight;
  return l;
}

}  // namespace

void launch_combine_lines(int64_t n_c, const LinePeaks &p0, const LinePeaks *p1, const LineOut &out, hipStream_t s) {
  if (n_c <= 0) {
    launch_fill_u64(reinterpret_cast<uint64_t *>(out.peak_offset), 1, 0, s);
    return;
  }
  const LineIn l0 = line_in(p0);
  const LineIn l1 = p1 ? line_in(*p1) : l0;
  hipLaunchKernelGGL(k_combine_lines, dim3((unsigned)n_c, kSplit), dim3(kThreads), 0, s, n_c, l0, l1, p1 != nullptr,
                     out);
}

}  // namespace xrd
