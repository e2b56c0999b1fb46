// Gaussian broadening of the reflections onto a 2theta grid, and the grid side
// of its adjoint.  The paper motivates fast simulation with machine-learning
// datasets of patterns modified by peak broadening (Section 1); this is the
// differentiable pattern those models consume.
//
//   y_g = sum_r I_r K(x_g - 2theta_r),  K(d) = exp(-d^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
//   restricted to |x_g - 2theta_r| <= window * sigma, x_g = t0 + g dt.
//
// Forward: a gather per grid point over the crystal's 2theta-sorted
// reflections (binary search for the window), summed in sorted order, so the
// result is deterministic without atomics.  Adjoint: per evaluated reflection,
// w1 = sum_g dL/dy_g K and w2 = sum_g dL/dy_g K (x_g - 2theta)/sigma^2 over the
// same window test.  Then the lattice chain rule of the per-crystal dL/dG*.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GridArgs {
  double t0, dt, sigma, half, norm, inv2s2;
  int64_t n;
};

__global__ __launch_bounds__(256) void k_broaden_fwd(const int64_t *__restrict__ refl_offset,
                                                     const double *__restrict__ skey,
                                                     const int32_t *__restrict__ sidx,
                                                     const double *__restrict__ inten, GridArgs g,
                                                     double *__restrict__ y) {
#pragma clang fp contract(off)
  const int64_t per = (g.n + 255) / 256;  // blocks per crystal
  const int64_t c = blockIdx.x / per;
  const int64_t gi = (int64_t)(blockIdx.x % per) * blockDim.x + threadIdx.x;
  if (gi >= g.n) return;
  const double x = g.t0 + (double)gi * g.dt;
  const int64_t r0 = refl_offset[c], r1 = refl_offset[c + 1];
  // first sorted position with 2theta >= x - half - guard; the exact window
  // test below decides, the guard only keeps rounding of the bound from
  // skipping a reflection the test would accept
  const double guard = 1e-9 * (fabs(x) + 1.0);
  const double lo = x - g.half - guard;
  int64_t a = r0, b = r1;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (skey[m] < lo) a = m + 1;
    else b = m;
  }
  double acc = 0.0;
  for (int64_t j = a; j < r1; ++j) {
    const double t = skey[j];
    const double d = x - t;
    if (t > x + g.half + guard) break;
    if (fabs(d) > g.half) continue;
    acc += inten[sidx[j]] * g.norm * exp(-(d * d) * g.inv2s2);
  }
  y[c * g.n + gi] = acc;
}

// Per evaluated reflection: w1 = sum dy K, w2 = sum dy K d / sigma^2 (d = x - 2theta).
__global__ __launch_bounds__(256) void k_broaden_adj(const SfItem *__restrict__ items, int64_t n_items,
                                                     bool friedel, const int64_t *__restrict__ refl_offset,
                                                     const double *__restrict__ tt, const double *__restrict__ dy,
                                                     GridArgs g, double *__restrict__ w1, double *__restrict__ w2) {
#pragma clang fp contract(off)
  const int64_t item = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (item >= n_items) return;
  const SfItem it = items[item];
  const int64_t r0 = refl_offset[it.crystal], r1 = refl_offset[it.crystal + 1];
  const int64_t first = friedel ? r0 + (r1 - r0) / 2 : r0;
  const int64_t count = friedel ? (r1 - r0) / 2 : r1 - r0;
  const int lane = threadIdx.x & 63;
  const double *dyc = dy + (int64_t)it.crystal * g.n;
  const double inv_s2 = 1.0 / (g.sigma * g.sigma);
  for (int u = 0; u < kSfRpt; ++u) {
    const int64_t e = (int64_t)it.tile * kSfTile + u * 64 + lane;
    if (e >= count) break;
    const int64_t i = first + e;
    const double t = tt[i];
    int64_t glo = (int64_t)floor((t - g.half - g.t0) / g.dt) - 1;
    int64_t ghi = (int64_t)ceil((t + g.half - g.t0) / g.dt) + 1;
    if (glo < 0) glo = 0;
    if (ghi > g.n - 1) ghi = g.n - 1;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t gi = glo; gi <= ghi; ++gi) {
      const double x = g.t0 + (double)gi * g.dt;
      const double d = x - t;
      if (fabs(d) > g.half) continue;
      const double kv = dyc[gi] * g.norm * exp(-(d * d) * g.inv2s2);
      a1 += kv;
      a2 += kv * d * inv_s2;
    }
    w1[i] = a1;
    w2[i] = a2;
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

void launch_broaden_fwd(int64_t n_c, const int64_t *refl_offset, const double *skey, const int32_t *sidx,
                        const double *inten, double t0, double dt, int64_t n, double sigma, double window,
                        double *y, hipStream_t s) {
  if (n_c <= 0 || n <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  hipLaunchKernelGGL(k_broaden_fwd, dim3((unsigned)(((n + 255) / 256) * n_c)), dim3(256), 0, s, refl_offset,
                     skey, sidx, inten, g, y);
}

void launch_broaden_adj(const SfItem *items, int64_t n_items, bool friedel, const int64_t *refl_offset,
                        const double *tt, const double *dy, double t0, double dt, int64_t n, double sigma,
                        double window, double *w1, double *w2, hipStream_t s) {
  if (n_items <= 0) return;
  const GridArgs g = make_grid(t0, dt, n, sigma, window);
  hipLaunchKernelGGL(k_broaden_adj, dim3((unsigned)((n_items + 3) / 4)), dim3(256), 0, s, items, n_items, friedel,
                     refl_offset, tt, dy, g, w1, w2);
}

void launch_lattice_chain(const CrystalPlan *plan, int64_t n_c, const double *part6, double *dlat, hipStream_t s) {
  if (n_c <= 0) return;
  hipLaunchKernelGGL(k_lattice_chain, dim3((unsigned)((n_c + 255) / 256)), dim3(256), 0, s, plan, n_c, part6, dlat);
}

}  // namespace xrd
